// Step a6: per-group interaction lists (Barnes' modified traversal with the
// cutoff pruning of the short-range part).
//
// One thread walks the preorder cell array for one group without a stack:
// a cell that is pruned, accepted or a leaf is left through its skip link,
// any other cell is opened by stepping to the next preorder index (its first
// child).  A count pass sizes the lists, a scan places them, and a write
// pass emits the entries in DFS order (particles ascending, cells in
// preorder).
//
// Compiled with -ffp-contract=off: the decisions are the literal FP64
// expressions, evaluated in this order:
//   per axis t = |cen_c - cen_g|, t = min(t, 1 - t), e = max(0, t - (half + h_g))
//   d2 = (e_x e_x + e_y e_y) + e_z e_z
//   prune  iff d2(half = side/2) >= r_cut * r_cut
//   accept iff side * side < (theta * theta) * d2(half = 0)
#include "common.h"

namespace srf {
namespace {

struct Frame {
    double cg[3], hg[3];
};

__device__ __forceinline__ Frame group_frame(const double* __restrict__ lo, const double* __restrict__ hi, int64_t g) {
    Frame f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double l = lo[g * 3 + a], h = hi[g * 3 + a];
        f.cg[a] = (l + h) * 0.5;
        f.hg[a] = (h - l) * 0.5;
    }
    return f;
}

__device__ __forceinline__ double axis_gap(double cen, double cg, double half) {
    double t = fabs(cen - cg);
    double t2 = 1.0 - t;
    t = t2 < t ? t2 : t;
    double r = t - half;
    return r > 0.0 ? r : 0.0;
}

// 0: pruned, 1: accepted as a monopole, 2: leaf (expand), 3: open.
__device__ __forceinline__ int classify(const NodeGeo& g, const Frame& f, double rc2, double th2) {
    const int lv = (int)(g.level_leaf & 0xffu);
    const double side = ldexp(1.0, -lv);
    const double hs = side * 0.5;
    const double cx = ldexp((double)g.ix + 0.5, -lv);
    const double cy = ldexp((double)g.iy + 0.5, -lv);
    const double cz = ldexp((double)g.iz + 0.5, -lv);
    double ex = axis_gap(cx, f.cg[0], hs + f.hg[0]);
    double ey = axis_gap(cy, f.cg[1], hs + f.hg[1]);
    double ez = axis_gap(cz, f.cg[2], hs + f.hg[2]);
    double D2 = (ex * ex + ey * ey) + ez * ez;
    if (D2 >= rc2) return 0;
    ex = axis_gap(cx, f.cg[0], f.hg[0]);
    ey = axis_gap(cy, f.cg[1], f.hg[1]);
    ez = axis_gap(cz, f.cg[2], f.hg[2]);
    double d2 = (ex * ex + ey * ey) + ez * ez;
    if (side * side < th2 * d2) return 1;
    if ((g.level_leaf >> 8) & 1u) return 2;
    return 3;
}

__global__ __launch_bounds__(128) void k_lists_count(int64_t ng, const double* __restrict__ glo,
                                                     const double* __restrict__ ghi, const int32_t* __restrict__ gcount,
                                                     const NodeGeo* __restrict__ geo, const NodeRange* __restrict__ rng,
                                                     int64_t nn, double rc2, double th2, int64_t* __restrict__ cnt,
                                                     unsigned long long* __restrict__ totals) {
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t np = 0, nc = 0;
    if (g < ng) {
        Frame f = group_frame(glo, ghi, g);
        int64_t i = 0;
        while (i < nn) {
            NodeGeo ge = geo[i];
            NodeRange r = rng[i];
            int k = classify(ge, f, rc2, th2);
            if (k == 3) {
                ++i;
                continue;
            }
            if (k == 1) ++nc;
            else if (k == 2) np += r.count;
            i = r.skip;
        }
        cnt[g] = np + nc;
    }
    // block sums of particle entries, cell entries and N_i * N_j
    unsigned long long a = (unsigned long long)np, b = (unsigned long long)nc;
    unsigned long long c = g < ng ? (unsigned long long)(gcount[g]) * (unsigned long long)(np + nc) : 0ull;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&totals[0], a);
        atomicAdd(&totals[1], b);
        atomicAdd(&totals[2], c);
    }
}

__global__ __launch_bounds__(128) void k_lists_write(int64_t ng, const double* __restrict__ glo,
                                                     const double* __restrict__ ghi, const NodeGeo* __restrict__ geo,
                                                     const NodeRange* __restrict__ rng, int64_t nn, double rc2,
                                                     double th2, const int64_t* __restrict__ off,
                                                     int32_t* __restrict__ ent) {
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= ng) return;
    Frame f = group_frame(glo, ghi, g);
    int32_t* out = ent + off[g];
    int64_t w = 0;
    int64_t i = 0;
    while (i < nn) {
        NodeGeo ge = geo[i];
        NodeRange r = rng[i];
        int k = classify(ge, f, rc2, th2);
        if (k == 3) {
            ++i;
            continue;
        }
        if (k == 1) {
            out[w++] = -(int32_t)i - 1;
        } else if (k == 2) {
            for (int32_t s = r.first; s < r.first + r.count; ++s) out[w++] = s;
        }
        i = r.skip;
    }
}

}  // namespace

void build_lists(const Tree& t, Lists& l, hipStream_t st) {
    const int64_t ng = t.n_groups;
    const double rc2 = l.r_cut * l.r_cut;
    const double th2 = l.theta * l.theta;
    l.n_groups = ng;
    l.off.alloc(ng + 1, st);
    DevBuf<unsigned long long> totals(4, st);
    SRF_HIP(hipMemsetAsync(totals.get(), 0, 4 * sizeof(unsigned long long), st));
    const int B = 128;
    hipLaunchKernelGGL(k_lists_count, dim3(grid_for(ng, B, 1 << 30)), dim3(B), 0, st, ng, t.glo.get(), t.ghi.get(),
                       t.gcount.get(), t.geo.get(), t.range.get(), t.n_nodes, rc2, th2, l.off.get(), totals.get());
    SRF_HIP(hipGetLastError());
    exclusive_scan_i64(l.off.get(), ng, true, st);
    unsigned long long h[3];
    SRF_HIP(hipMemcpyAsync(h, totals.get(), 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SRF_HIP(hipStreamSynchronize(st));
    l.n_particle_entries = (int64_t)h[0];
    l.n_node_entries = (int64_t)h[1];
    l.n_entries = (int64_t)(h[0] + h[1]);
    l.interactions = (int64_t)h[2];
    l.ent.alloc(l.n_entries > 0 ? l.n_entries : 1, st);
    hipLaunchKernelGGL(k_lists_write, dim3(grid_for(ng, B, 1 << 30)), dim3(B), 0, st, ng, t.glo.get(), t.ghi.get(),
                       t.geo.get(), t.range.get(), t.n_nodes, rc2, th2, l.off.get(), l.ent.get());
    SRF_HIP(hipGetLastError());
}

}  // namespace srf
