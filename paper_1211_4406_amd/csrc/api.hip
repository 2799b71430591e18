// The C ABI (include/srf.h): validation, handles, error codes, export.
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

struct srf_tree {
    srf::Tree t;
};
struct srf_lists {
    srf::Lists l;
};

namespace {

thread_local std::string g_last_error;

// Tree generation numbers: a tree freed and another built at the same
// address still gets a new number, so stale lists are refused.
std::atomic<uint64_t> g_tree_generation{0};

int set_error(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

template <class F>
int guarded(F&& f) {
    try {
        f();
        return SRF_OK;
    } catch (const srf::Error& e) {
        return set_error(e.status, e.msg);
    } catch (const std::bad_alloc&) {
        return set_error(SRF_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_error(SRF_EHIP, "unexpected internal error");
    }
}

void validate(const srf_params* p) {
    if (!p) srf::fail(SRF_EINVAL, "params is NULL");
    if (!std::isfinite(p->G)) srf::fail(SRF_EINVAL, "G must be finite");
    if (!(std::isfinite(p->r_cut) && p->r_cut > 0.0 && p->r_cut < 0.25))
        srf::fail(SRF_EINVAL, "r_cut must lie in (0, 0.25)");
    if (!(std::isfinite(p->eps) && p->eps > 0.0)) srf::fail(SRF_EINVAL, "eps must be finite and > 0");
    if (!(std::isfinite(p->theta) && p->theta >= 0.0 && p->theta <= 1.0))
        srf::fail(SRF_EINVAL, "theta must lie in [0, 1]");
    if (p->n_group < 1 || p->n_group > 64) srf::fail(SRF_EINVAL, "n_group must lie in [1, 64]");
    if (p->n_leaf < 1 || p->n_leaf > p->n_group) srf::fail(SRF_EINVAL, "n_leaf must lie in [1, n_group]");
    if (p->precision != SRF_FP32_REL && p->precision != SRF_FP64) srf::fail(SRF_EINVAL, "unknown precision");
    if (p->compensated != 0 && p->compensated != 1) srf::fail(SRF_EINVAL, "compensated must be 0 or 1");
    if (p->mac != SRF_MAC_CENTRE && p->mac != SRF_MAC_COM) srf::fail(SRF_EINVAL, "unknown mac");
}

void check_pair(const srf_tree* t, const srf_lists* l, const srf_params* p) {
    if (!t || !l) srf::fail(SRF_EINVAL, "tree or lists is NULL");
    validate(p);
    if (l->l.tree_id != t->t.id) srf::fail(SRF_EMISMATCH, "lists were built from another tree");
    if (p->r_cut != l->l.r_cut || p->theta != l->l.theta || p->mac != l->l.mac || p->n_group != t->t.n_group ||
        p->n_leaf != t->t.n_leaf)
        srf::fail(SRF_EMISMATCH, "params differ from those the tree and lists were built with");
}

struct Timing {
    bool enabled = false;
    bool have[3] = {false, false, false};
    hipEvent_t ev[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
};
Timing g_timing;

void timing_events(int which, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!g_timing.enabled) return;
    if (!g_timing.ev[which][0]) {
        SRF_HIP(hipEventCreate(&g_timing.ev[which][0]));
        SRF_HIP(hipEventCreate(&g_timing.ev[which][1]));
    }
    *e0 = g_timing.ev[which][0];
    *e1 = g_timing.ev[which][1];
    g_timing.have[which] = true;
}

template <class S, class D>
void copy_out(D* host, const S* dev, int64_t count, hipStream_t st) {
    if (!host || count <= 0) return;
    std::vector<S> tmp(count);
    SRF_HIP(hipMemcpyAsync(tmp.data(), dev, count * sizeof(S), hipMemcpyDeviceToHost, st));
    SRF_HIP(hipStreamSynchronize(st));
    for (int64_t i = 0; i < count; ++i) host[i] = (D)tmp[i];
}

}  // namespace

extern "C" {

int srf_tree_build(int64_t n, const double* x, const double* y, const double* z, int64_t pos_stride, const double* m,
                   int64_t m_stride, const srf_params* p, void* stream, srf_tree** out) {
    if (out) *out = nullptr;
    srf_tree* h = nullptr;
    int rc = guarded([&] {
        validate(p);
        if (!out) srf::fail(SRF_EINVAL, "out is NULL");
        if (n < 1 || n >= (int64_t)0x7fffffff - 1) srf::fail(SRF_EINVAL, "n must lie in [1, 2^31 - 2)");
        if (!x || !y || !z || !m) srf::fail(SRF_EINVAL, "NULL position or mass pointer");
        if (pos_stride < 1 || m_stride < 1) srf::fail(SRF_EINVAL, "strides must be >= 1");
        hipStream_t st = (hipStream_t)stream;
        h = new srf_tree();
        srf::Tree& t = h->t;
        t.id = ++g_tree_generation;
        t.n = n;
        t.n_group = p->n_group;
        t.n_leaf = p->n_leaf;
        t.stream = st;
        srf::DevBuf<int32_t> flag(1, st);
        srf::fill_i32(flag.get(), 0, 1, st);
        srf::build_sorted(t, x, y, z, pos_stride, m, m_stride, flag.get(), false, st);
        // reads the flag at its one synchronisation (SRF_EDOMAIN); when more
        // particles than the run sort takes share one high key word (a dense
        // clump in a 2^-10 cube), the tree is built again on the full sort
        if (!srf::build_cells_and_groups(t, flag.get(), st)) {
            srf::fill_i32(flag.get(), 0, 1, st);
            srf::build_sorted(t, x, y, z, pos_stride, m, m_stride, flag.get(), true, st);
            if (!srf::build_cells_and_groups(t, flag.get(), st))
                srf::fail(SRF_EHIP, "the full radix sort reported an incomplete order");
        }
    });
    if (rc != SRF_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return SRF_OK;
}

int srf_tree_refit(srf_tree* t, const double* x, const double* y, const double* z, int64_t pos_stride,
                   const double* m, int64_t m_stride, void* stream) {
    return guarded([&] {
        if (!t) srf::fail(SRF_EINVAL, "tree is NULL");
        if (!x || !y || !z) srf::fail(SRF_EINVAL, "NULL position pointer");
        if (pos_stride < 1 || (m && m_stride < 1)) srf::fail(SRF_EINVAL, "strides must be >= 1");
        srf::Tree& T = t->t;
        hipStream_t st = (hipStream_t)stream;
        const int64_t n = T.n;
        // gather into new buffers: the tree is untouched until the inputs pass
        srf::DevBuf<double> nx(n, st), ny(n, st), nz(n, st), nm;
        if (m) nm.alloc(n, st);
        srf::DevBuf<int32_t> flag(1, st);
        srf::fill_i32(flag.get(), 0, 1, st);
        srf::gather_refit(T, x, y, z, pos_stride, m, m_stride, flag.get(), nx.get(), ny.get(), nz.get(),
                          m ? nm.get() : nullptr, st);
        int32_t hflag = 0;
        SRF_HIP(hipMemcpyAsync(&hflag, flag.get(), sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SRF_HIP(hipStreamSynchronize(st));
        if (hflag & 1) srf::fail(SRF_EDOMAIN, "non-finite particle position");
        if (hflag & 2) srf::fail(SRF_EDOMAIN, "particle mass not finite and > 0");
        T.px = std::move(nx);
        T.py = std::move(ny);
        T.pz = std::move(nz);
        if (m) T.pm = std::move(nm);
        T.id = ++g_tree_generation;   // lists of the old positions are refused from here on
        T.refit = true;
        srf::refit_cells_and_groups(T, st);
    });
}

int srf_make_lists(const srf_tree* t, const srf_params* p, void* stream, srf_lists** out) {
    if (out) *out = nullptr;
    srf_lists* h = nullptr;
    int rc = guarded([&] {
        validate(p);
        if (!t || !out) srf::fail(SRF_EINVAL, "NULL tree or out");
        if (p->n_group != t->t.n_group || p->n_leaf != t->t.n_leaf)
            srf::fail(SRF_EMISMATCH, "n_group / n_leaf differ from the tree's");
        hipStream_t st = (hipStream_t)stream;
        h = new srf_lists();
        srf::Lists& l = h->l;
        l.tree_id = t->t.id;
        l.r_cut = p->r_cut;
        l.theta = p->theta;
        l.mac = p->mac;
        l.n_group = p->n_group;
        l.n_leaf = p->n_leaf;
        l.stream = st;
        srf::build_lists(t->t, l, st);
    });
    if (rc != SRF_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return SRF_OK;
}

int srf_short_range_force(const srf_tree* t, const srf_lists* l, const srf_params* p, double* ax, double* ay,
                          double* az, int64_t out_stride, void* stream) {
    return guarded([&] {
        check_pair(t, l, p);
        if (!ax || !ay || !az) srf::fail(SRF_EINVAL, "NULL output pointer");
        if (out_stride < 1) srf::fail(SRF_EINVAL, "out_stride must be >= 1");
        hipEvent_t e0, e1;
        timing_events(0, &e0, &e1);
        srf::launch_force(t->t, l->l, *p, ax, ay, az, out_stride, (hipStream_t)stream, e0, e1);
    });
}

int srf_short_range_adjoint(const srf_tree* t, const srf_lists* l, const srf_params* p, const double* wx,
                            const double* wy, const double* wz, int64_t w_stride, double* gx, double* gy, double* gz,
                            int64_t g_stride, double* gm, int64_t gm_stride, void* stream) {
    return guarded([&] {
        check_pair(t, l, p);
        if (!wx || !wy || !wz || !gx || !gy || !gz || !gm) srf::fail(SRF_EINVAL, "NULL pointer");
        if (w_stride < 1 || g_stride < 1 || gm_stride < 1) srf::fail(SRF_EINVAL, "strides must be >= 1");
        if (t->t.n + t->t.n_nodes > INT32_MAX)
            srf::fail(SRF_EINVAL, "the adjoint indexes particles and cells with 32-bit rows: n + n_cells too large");
        hipEvent_t e0, e1;
        timing_events(1, &e0, &e1);
        srf::launch_adjoint(t->t, l->l, *p, wx, wy, wz, w_stride, gx, gy, gz, g_stride, gm, gm_stride,
                            (hipStream_t)stream, e0, e1);
    });
}

int srf_short_range_adjoint_noalloc(const srf_tree* t, const srf_lists* l, const srf_params* p, const double* wx,
                                    const double* wy, const double* wz, int64_t w_stride, double* gx, double* gy,
                                    double* gz, int64_t g_stride, double* gm, int64_t gm_stride, void* stream) {
    return guarded([&] {
        check_pair(t, l, p);
        if (!wx || !wy || !wz || !gx || !gy || !gz || !gm) srf::fail(SRF_EINVAL, "NULL pointer");
        if (w_stride < 1 || g_stride < 1 || gm_stride < 1) srf::fail(SRF_EINVAL, "strides must be >= 1");
        if (t->t.n + t->t.n_nodes > INT32_MAX)
            srf::fail(SRF_EINVAL, "the adjoint indexes particles and cells with 32-bit rows: n + n_cells too large");
        srf::launch_adjoint_noalloc(t->t, l->l, *p, wx, wy, wz, w_stride, gx, gy, gz, g_stride, gm, gm_stride,
                                    (hipStream_t)stream);
    });
}

int srf_short_range_quadrupole(const srf_tree* t, const srf_lists* l, const srf_params* p, double* ax, double* ay,
                               double* az, int64_t out_stride, void* stream) {
    return guarded([&] {
        check_pair(t, l, p);
        if (!ax || !ay || !az) srf::fail(SRF_EINVAL, "NULL output pointer");
        if (out_stride < 1) srf::fail(SRF_EINVAL, "out_stride must be >= 1");
        srf::launch_quadrupole(t->t, l->l, *p, ax, ay, az, out_stride, (hipStream_t)stream);
    });
}

int srf_short_range_potential(const srf_tree* t, const srf_lists* l, const srf_params* p, double* phi,
                              int64_t out_stride, void* stream) {
    return guarded([&] {
        check_pair(t, l, p);
        if (!phi) srf::fail(SRF_EINVAL, "NULL output pointer");
        if (out_stride < 1) srf::fail(SRF_EINVAL, "out_stride must be >= 1");
        if (t->t.n + t->t.n_nodes > INT32_MAX)
            srf::fail(SRF_EINVAL, "the potential indexes particles and cells with 32-bit rows: n + n_cells too large");
        srf::launch_potential(t->t, l->l, *p, phi, out_stride, (hipStream_t)stream);
    });
}

int srf_pm_force(const srf_tree* t, double G, double r_cut, int32_t n_mesh, double* ax, double* ay, double* az,
                 int64_t out_stride, void* stream) {
    return guarded([&] {
        if (!t) srf::fail(SRF_EINVAL, "tree is NULL");
        if (!ax || !ay || !az) srf::fail(SRF_EINVAL, "NULL output pointer");
        if (out_stride < 1) srf::fail(SRF_EINVAL, "out_stride must be >= 1");
        if (!std::isfinite(G)) srf::fail(SRF_EINVAL, "G must be finite");
        if (!(std::isfinite(r_cut) && r_cut > 0.0 && r_cut < 0.25)) srf::fail(SRF_EINVAL, "r_cut must lie in (0, 0.25)");
        if (n_mesh < 16 || n_mesh > 1024 || (n_mesh & (n_mesh - 1)) != 0)
            srf::fail(SRF_EINVAL, "n_mesh must be a power of two in [16, 1024]");
        hipEvent_t e0, e1;
        timing_events(2, &e0, &e1);
        srf::launch_pm(t->t, G, r_cut, n_mesh, ax, ay, az, out_stride, (hipStream_t)stream, e0, e1);
    });
}

int srf_kick(int64_t n, double* vx, double* vy, double* vz, int64_t v_stride, const double* ax, const double* ay,
             const double* az, int64_t a_stride, double dt, void* stream) {
    return guarded([&] {
        if (n < 1) srf::fail(SRF_EINVAL, "n must be >= 1");
        if (!vx || !vy || !vz || !ax || !ay || !az) srf::fail(SRF_EINVAL, "NULL pointer");
        if (v_stride < 1 || a_stride < 1) srf::fail(SRF_EINVAL, "strides must be >= 1");
        if (!std::isfinite(dt)) srf::fail(SRF_EINVAL, "dt must be finite");
        srf::launch_kick(n, vx, vy, vz, v_stride, ax, ay, az, a_stride, dt, (hipStream_t)stream);
    });
}

int srf_drift(int64_t n, double* x, double* y, double* z, int64_t x_stride, const double* vx, const double* vy,
              const double* vz, int64_t v_stride, double dt, void* stream) {
    return guarded([&] {
        if (n < 1) srf::fail(SRF_EINVAL, "n must be >= 1");
        if (!x || !y || !z || !vx || !vy || !vz) srf::fail(SRF_EINVAL, "NULL pointer");
        if (x_stride < 1 || v_stride < 1) srf::fail(SRF_EINVAL, "strides must be >= 1");
        if (!std::isfinite(dt)) srf::fail(SRF_EINVAL, "dt must be finite");
        srf::launch_drift(n, x, y, z, x_stride, vx, vy, vz, v_stride, dt, (hipStream_t)stream);
    });
}

void srf_tree_free(srf_tree* t) { delete t; }
void srf_lists_free(srf_lists* l) { delete l; }
void srf_release_cache(void) { srf::dev_release_all(); }

const char* srf_strerror(int status) {
    switch (status) {
        case SRF_OK: return "success";
        case SRF_EINVAL: return "invalid argument";
        case SRF_EDOMAIN: return "invalid particle data (non-finite position or mass <= 0)";
        case SRF_ENOMEM: return "out of device memory";
        case SRF_EHIP: return "HIP runtime error";
        case SRF_EMISMATCH: return "tree, lists and parameters do not match";
        default: return "unknown status";
    }
}

const char* srf_last_error(void) { return g_last_error.c_str(); }

int srf_tree_info(const srf_tree* t, int64_t* n, int64_t* n_nodes, int64_t* n_groups, int32_t* max_level) {
    return guarded([&] {
        if (!t) srf::fail(SRF_EINVAL, "tree is NULL");
        if (n) *n = t->t.n;
        if (n_nodes) *n_nodes = t->t.n_nodes;
        if (n_groups) *n_groups = t->t.n_groups;
        if (max_level) *max_level = t->t.max_level;
    });
}

int srf_tree_export(const srf_tree* t, uint64_t* keys_sorted, int64_t* perm, int32_t* node_level,
                    uint64_t* node_prefix, int64_t* node_first, int64_t* node_count, int64_t* group_first,
                    int64_t* group_count, double* group_lo, double* group_hi) {
    return guarded([&] {
        if (!t) srf::fail(SRF_EINVAL, "tree is NULL");
        const srf::Tree& T = t->t;
        hipStream_t st = T.stream;
        copy_out(keys_sorted, T.keys.get(), T.n, st);
        copy_out(perm, T.perm.get(), T.n, st);
        copy_out(node_prefix, T.prefix.get(), T.n_nodes, st);
        copy_out(group_first, T.gfirst.get(), T.n_groups, st);
        copy_out(group_count, T.gcount.get(), T.n_groups, st);
        copy_out(group_lo, T.glo.get(), T.n_groups * 3, st);
        copy_out(group_hi, T.ghi.get(), T.n_groups * 3, st);
        if (node_level || node_first || node_count) {
            std::vector<srf::NodeGeo> geo(T.n_nodes);
            std::vector<srf::NodeRange> rng(T.n_nodes);
            SRF_HIP(hipMemcpyAsync(geo.data(), T.geo.get(), T.n_nodes * sizeof(srf::NodeGeo), hipMemcpyDeviceToHost, st));
            SRF_HIP(hipMemcpyAsync(rng.data(), T.range.get(), T.n_nodes * sizeof(srf::NodeRange), hipMemcpyDeviceToHost,
                                   st));
            SRF_HIP(hipStreamSynchronize(st));
            for (int64_t c = 0; c < T.n_nodes; ++c) {
                if (node_level) node_level[c] = (int32_t)(geo[c].level_leaf & 0xffu);
                if (node_first) node_first[c] = rng[c].first;
                if (node_count) node_count[c] = rng[c].count;
            }
        }
    });
}

int srf_moments_export(const srf_tree* t, double* M, double* X, double* Y, double* Z) {
    return guarded([&] {
        if (!t) srf::fail(SRF_EINVAL, "tree is NULL");
        const srf::Tree& T = t->t;
        copy_out(M, T.nM.get(), T.n_nodes, T.stream);
        copy_out(X, T.nX.get(), T.n_nodes, T.stream);
        copy_out(Y, T.nY.get(), T.n_nodes, T.stream);
        copy_out(Z, T.nZ.get(), T.n_nodes, T.stream);
    });
}

int srf_cell_boxes_export(const srf_tree* t, double* lo, double* hi) {
    return guarded([&] {
        if (!t) srf::fail(SRF_EINVAL, "tree is NULL");
        const srf::Tree& T = t->t;
        if (!T.refit) srf::fail(SRF_EINVAL, "the tree has not been refitted: its cells are their dyadic boxes");
        copy_out(lo, T.clo.get(), T.n_nodes * 3, T.stream);
        copy_out(hi, T.chi.get(), T.n_nodes * 3, T.stream);
    });
}

int srf_sorted_export(const srf_tree* t, double* x, double* y, double* z, double* m) {
    return guarded([&] {
        if (!t) srf::fail(SRF_EINVAL, "tree is NULL");
        const srf::Tree& T = t->t;
        copy_out(x, T.px.get(), T.n, T.stream);
        copy_out(y, T.py.get(), T.n, T.stream);
        copy_out(z, T.pz.get(), T.n, T.stream);
        copy_out(m, T.pm.get(), T.n, T.stream);
    });
}

int srf_lists_info(const srf_lists* l, int64_t* n_groups, int64_t* n_particle_entries, int64_t* n_node_entries,
                   int64_t* interactions) {
    return guarded([&] {
        if (!l) srf::fail(SRF_EINVAL, "lists is NULL");
        if (n_groups) *n_groups = l->l.n_groups;
        if (n_particle_entries) *n_particle_entries = l->l.n_particle_entries;
        if (n_node_entries) *n_node_entries = l->l.n_node_entries;
        if (interactions) *interactions = l->l.interactions;
    });
}

int srf_lists_export(const srf_lists* l, int64_t* poff, int64_t* pidx, int64_t* noff, int64_t* nidx) {
    return guarded([&] {
        if (!l) srf::fail(SRF_EINVAL, "lists is NULL");
        const srf::Lists& L = l->l;
        std::vector<int64_t> off(L.n_groups + 1);
        std::vector<int32_t> ent(L.n_entries);
        hipStream_t st = L.stream;
        SRF_HIP(hipMemcpyAsync(off.data(), L.off.get(), (L.n_groups + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        if (L.n_entries > 0)
            SRF_HIP(hipMemcpyAsync(ent.data(), L.ent.get(), L.n_entries * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        SRF_HIP(hipStreamSynchronize(st));
        int64_t wp = 0, wn = 0;
        for (int64_t g = 0; g < L.n_groups; ++g) {
            if (poff) poff[g] = wp;
            if (noff) noff[g] = wn;
            for (int64_t e = off[g]; e < off[g + 1]; ++e) {
                const int32_t v = ent[e];
                if (v >= 0) {
                    if (pidx) pidx[wp] = v;
                    ++wp;
                } else {
                    if (nidx) nidx[wn] = -(int64_t)v - 1;
                    ++wn;
                }
            }
        }
        if (poff) poff[L.n_groups] = wp;
        if (noff) noff[L.n_groups] = wn;
    });
}

int srf_set_kernel_timing(int enable) {
    g_timing.enabled = enable != 0;
    return SRF_OK;
}

int srf_last_kernel_ms(const char* which, double* ms) {
    return guarded([&] {
        if (!which || !ms) srf::fail(SRF_EINVAL, "NULL argument");
        int k = std::strcmp(which, "force") == 0 ? 0
                : std::strcmp(which, "adjoint") == 0 ? 1
                : std::strcmp(which, "pm") == 0      ? 2
                                                     : -1;
        if (k < 0) srf::fail(SRF_EINVAL, "which must be \"force\", \"adjoint\" or \"pm\"");
        if (!g_timing.have[k]) srf::fail(SRF_EINVAL, "no timed launch recorded");
        SRF_HIP(hipEventSynchronize(g_timing.ev[k][1]));
        float f = 0.0f;
        SRF_HIP(hipEventElapsedTime(&f, g_timing.ev[k][0], g_timing.ev[k][1]));
        *ms = f;
    });
}

}  // extern "C"
