// Steps a3-a5: octree over the Morton order (built level by level), monopole
// moments (bottom-up), renumbering into DFS preorder with subtree "skip"
// links, particle groups and their bounding boxes.
//
// Compiled with -ffp-contract=off: the group boxes feed the list decisions,
// which must be the literal FP64 expressions.
#include <algorithm>
#include <vector>

#include "common.h"

namespace srf {
namespace {

// Breadth-first cell arrays used while building (level-major order).
struct Bfs {
    int64_t cap = 0;
    DevBuf<int32_t> level, first, count, parent, child_begin, child_cnt;
    DevBuf<uint64_t> prefix;
};

void bfs_alloc(Bfs& b, int64_t cap, hipStream_t st) {
    b.cap = cap;
    b.level.alloc(cap, st);
    b.first.alloc(cap, st);
    b.count.alloc(cap, st);
    b.parent.alloc(cap, st);
    b.child_begin.alloc(cap, st);
    b.child_cnt.alloc(cap, st);
    b.prefix.alloc(cap, st);
}

template <class T>
void grow_one(DevBuf<T>& buf, int64_t used, int64_t cap, hipStream_t st) {
    DevBuf<T> nb(cap, st);
    if (used > 0) SRF_HIP(hipMemcpyAsync(nb.get(), buf.get(), used * sizeof(T), hipMemcpyDeviceToDevice, st));
    buf = std::move(nb);
}

void bfs_grow(Bfs& b, int64_t used, int64_t need, hipStream_t st) {
    if (need <= b.cap) return;
    int64_t cap = std::max<int64_t>(need, b.cap * 2);
    grow_one(b.level, used, cap, st);
    grow_one(b.first, used, cap, st);
    grow_one(b.count, used, cap, st);
    grow_one(b.parent, used, cap, st);
    grow_one(b.child_begin, used, cap, st);
    grow_one(b.child_cnt, used, cap, st);
    grow_one(b.prefix, used, cap, st);
    b.cap = cap;
}

__global__ void k_root(int64_t n, int32_t* level, int32_t* first, int32_t* count, int32_t* parent,
                       uint64_t* prefix) {
    level[0] = 0;
    first[0] = 0;
    count[0] = (int32_t)n;
    parent[0] = -1;
    prefix[0] = 0;
}

// First index in [lo, hi) whose level-(L+1) digit is >= o (digits are
// non-decreasing inside a cell).
__device__ __forceinline__ int32_t lower_digit(const uint64_t* __restrict__ keys, int32_t lo, int32_t hi, int shift,
                                               uint32_t o) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        uint32_t dg = (uint32_t)((keys[mid] >> shift) & 7u);
        if (dg < o) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Children of the cells of one level: octant boundaries and counts.  Eight
// threads per cell (32 cells per block of 256): thread o finds boundary o
// (the first index whose level-(L+1) digit is >= o; o = 0 is the cell's
// first index), so each thread's chain of dependent loads is one binary
// search; thread 0 then counts the non-empty octants.
__global__ __launch_bounds__(256) void k_child_count(int64_t begin, int64_t m, int level, int32_t n_leaf,
                                                     const int32_t* __restrict__ first,
                                                     const int32_t* __restrict__ count,
                                                     const uint64_t* __restrict__ keys, int32_t* __restrict__ bnd,
                                                     int32_t* __restrict__ cnt) {
    __shared__ int32_t sb[256 + 32];
    const int64_t k = blockIdx.x * 32ll + (threadIdx.x >> 3);
    const int o = threadIdx.x & 7;
    const int slot = (threadIdx.x >> 3) * 9;
    bool split = false;
    if (k < m) {
        const int64_t c = begin + k;
        const int32_t f = first[c], nc = count[c];
        split = (level == 0) || (level < kMaxLevel && nc > n_leaf);
        if (split) {
            const int shift = 3 * (kMaxLevel - (level + 1));
            const int32_t bo = o == 0 ? f : lower_digit(keys, f, f + nc, shift, (uint32_t)o);
            sb[slot + o] = bo;
            bnd[k * 9 + o] = bo;
            if (o == 0) {
                sb[slot + 8] = f + nc;
                bnd[k * 9 + 8] = f + nc;
            }
        }
    }
    __syncthreads();
    if (k < m && o == 0) {
        int nz = 0;
        if (split) {
#pragma unroll
            for (int q = 0; q < 8; ++q) nz += (sb[slot + q + 1] > sb[slot + q]) ? 1 : 0;
        }
        cnt[k] = nz;
    }
}

__global__ void k_child_write(int64_t begin, int64_t m, int64_t out_begin, int level, const int32_t* __restrict__ bnd,
                              const int32_t* __restrict__ off, int32_t* __restrict__ lv, int32_t* __restrict__ first,
                              int32_t* __restrict__ count, int32_t* __restrict__ parent,
                              int32_t* __restrict__ child_begin, int32_t* __restrict__ child_cnt,
                              uint64_t* __restrict__ prefix) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    int64_t c = begin + k;
    int32_t nz = off[k + 1] - off[k];
    int64_t out = out_begin + off[k];
    child_begin[c] = (int32_t)out;
    child_cnt[c] = nz;
    if (nz == 0) return;
    const int32_t* b = bnd + k * 9;
    uint64_t pp = prefix[c];
    for (int o = 0; o < 8; ++o) {
        int32_t cc = b[o + 1] - b[o];
        if (cc <= 0) continue;
        lv[out] = level + 1;
        first[out] = b[o];
        count[out] = cc;
        parent[out] = (int32_t)c;
        prefix[out] = pp * 8u + (uint64_t)o;
        ++out;
    }
}

__global__ void k_leaf_fix(int64_t begin, int64_t m, int32_t* __restrict__ child_begin, int32_t* __restrict__ child_cnt) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= m) return;
    child_begin[begin + k] = -1;
    child_cnt[begin + k] = 0;
}

// Bottom-up monopoles of one level: mass and mass-weighted position sums,
// 4 lanes per cell.  A leaf's lane j takes its particles j, j + 4, ...
// (consecutive lanes read consecutive particles), an inner cell's lane j
// its children j, j + 4.  The 4 partial sums are then added by shuffles.
constexpr int kMomLanes = 4;

__global__ __launch_bounds__(256) void k_moments(int64_t begin, int64_t m, const int32_t* __restrict__ first,
                                                 const int32_t* __restrict__ count,
                                                 const int32_t* __restrict__ child_begin,
                                                 const int32_t* __restrict__ child_cnt, const double* __restrict__ px,
                                                 const double* __restrict__ py, const double* __restrict__ pz,
                                                 const double* __restrict__ pm, double* __restrict__ M,
                                                 double* __restrict__ SX, double* __restrict__ SY,
                                                 double* __restrict__ SZ) {
    const int64_t k = blockIdx.x * (int64_t)(256 / kMomLanes) + threadIdx.x / kMomLanes;
    const int j = threadIdx.x & (kMomLanes - 1);
    const bool on = k < m;
    const int64_t c = begin + (on ? k : 0);
    double sm = 0, sx = 0, sy = 0, sz = 0;
    if (on) {
        const int32_t nch = child_cnt[c];
        if (nch == 0) {
            const int32_t f = first[c], e = first[c] + count[c];
            for (int32_t s = f + j; s < e; s += kMomLanes) {
                const double mm = pm[s];
                sm += mm;
                sx += mm * px[s];
                sy += mm * py[s];
                sz += mm * pz[s];
            }
        } else {
            const int32_t cb = child_begin[c];
            for (int32_t q = cb + j; q < cb + nch; q += kMomLanes) {
                sm += M[q];
                sx += SX[q];
                sy += SY[q];
                sz += SZ[q];
            }
        }
    }
#pragma unroll
    for (int o = kMomLanes / 2; o >= 1; o >>= 1) {
        sm += __shfl_xor(sm, o, kMomLanes);
        sx += __shfl_xor(sx, o, kMomLanes);
        sy += __shfl_xor(sy, o, kMomLanes);
        sz += __shfl_xor(sz, o, kMomLanes);
    }
    if (on && j == 0) {
        M[c] = sm;
        SX[c] = sx;
        SY[c] = sy;
        SZ[c] = sz;
    }
}

// Preorder numbering: the cells starting at sorted index f form one chain
// of consecutive levels (each the first child of the previous), so
// pre(c) = start[f] + level(c) - minlevel(f), with start[] the exclusive
// scan of the number of cells starting at each index.  Every chain ends in
// the leaf that starts at f, so each leaf walks up its chain (while the
// parent starts at the same index) and stores the chain's length and top
// level: one plain store per index, no atomics.
__global__ void k_pre_count(int64_t nn, const int32_t* __restrict__ first, const int32_t* __restrict__ level,
                            const int32_t* __restrict__ parent, const int32_t* __restrict__ child_cnt,
                            int32_t* __restrict__ cntf, int32_t* __restrict__ minlv) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nn || child_cnt[c] != 0) return;
    const int32_t f = first[c];
    int32_t top = level[c];
    int32_t p = parent[c];
    while (p >= 0 && first[p] == f) {
        top = level[p];
        p = parent[p];
    }
    cntf[f] = level[c] - top + 1;
    minlv[f] = top;
}

__global__ void k_pre_assign(int64_t nn, const int32_t* __restrict__ first, const int32_t* __restrict__ level,
                             const int32_t* __restrict__ start, const int32_t* __restrict__ minlv,
                             int32_t* __restrict__ bfs2pre) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nn) return;
    int32_t f = first[c];
    bfs2pre[c] = start[f] + level[c] - minlv[f];
}

__device__ __forceinline__ uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

__global__ void k_pre_scatter(int64_t nn, int64_t n, const int32_t* __restrict__ bfs2pre,
                              const int32_t* __restrict__ level, const int32_t* __restrict__ first,
                              const int32_t* __restrict__ count, const int32_t* __restrict__ parent,
                              const int32_t* __restrict__ child_cnt, const uint64_t* __restrict__ prefix,
                              const int32_t* __restrict__ start, const double* __restrict__ M,
                              const double* __restrict__ SX, const double* __restrict__ SY,
                              const double* __restrict__ SZ, NodeGeo* __restrict__ geo, NodeRange* __restrict__ rng,
                              uint4* __restrict__ pack,
                              uint64_t* __restrict__ opre, double* __restrict__ oM, double* __restrict__ oX,
                              double* __restrict__ oY, double* __restrict__ oZ, int32_t* __restrict__ leaf_of) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nn) return;
    int32_t p = bfs2pre[c];
    uint64_t pf = prefix[c];
    int32_t lv = level[c];
    bool leaf = child_cnt[c] == 0;
    NodeGeo g;
    g.ix = compact3(pf >> 2);
    g.iy = compact3(pf >> 1);
    g.iz = compact3(pf);
    g.level_leaf = (uint32_t)lv | (leaf ? 0x100u : 0u);
    geo[p] = g;
    int32_t f = first[c], cnt = count[c];
    NodeRange r;
    r.first = f;
    r.count = cnt;
    r.skip = start[f + cnt];
    r.parent = parent[c] >= 0 ? bfs2pre[parent[c]] : -1;
    rng[p] = r;
    const uint32_t sk = (uint32_t)r.skip;
    uint4 pk;
    pk.x = g.ix | ((sk & 0x7ffu) << 21);
    pk.y = g.iy | (((sk >> 11) & 0x7ffu) << 21);
    pk.z = g.iz | (((sk >> 22) & 0x3ffu) << 21);
    pk.w = (uint32_t)lv | (leaf ? 0x20u : 0u) | ((uint32_t)(cnt < (int32_t)kPackCountMax ? cnt : (int32_t)kPackCountMax) << 6);
    pack[p] = pk;
    opre[p] = pf;
    double mm = M[c];
    oM[p] = mm;
    oX[p] = SX[c] / mm;
    oY[p] = SY[c] / mm;
    oZ[p] = SZ[c] / mm;
    if (leaf)
        for (int32_t s = f; s < f + cnt; ++s) leaf_of[s] = p;
    (void)n;
}

// Group starts.  A "group parent" is the root or a cell with more than
// n_group particles.  Its candidate children (at most n_group particles)
// start groups: each on its own under the root, merged greedily with the
// following candidate siblings (in octant order) otherwise.  A level-21
// cell with more than n_group particles is cut into chunks of n_group.
__global__ void k_group_marks(int64_t nn, int32_t n_g, const NodeGeo* __restrict__ geo,
                              const NodeRange* __restrict__ rng, int32_t* __restrict__ mark) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nn) return;
    NodeRange r = rng[c];
    int lv = (int)(geo[c].level_leaf & 0xffu);
    if (!(lv == 0 || r.count > n_g)) return;
    bool leaf = (geo[c].level_leaf >> 8) & 1u;
    if (leaf) {  // level 21, too many coincident keys
        for (int32_t s = 0; s < r.count; s += n_g) mark[r.first + s] = 1;
        return;
    }
    bool merge = lv >= 1;
    bool open = false;
    int32_t run = 0;
    int32_t ch = (int32_t)c + 1;
    while (ch < r.skip) {
        NodeRange q = rng[ch];
        if (q.count <= n_g) {
            if (merge && open && run + q.count <= n_g) {
                run += q.count;
            } else {
                mark[q.first] = 1;
                open = true;
                run = q.count;
            }
        } else {
            open = false;
            run = 0;
        }
        ch = q.skip;
    }
}

__global__ void k_group_write(int64_t n, const int32_t* __restrict__ sc, int32_t* __restrict__ gfirst) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    if (sc[s + 1] != sc[s]) gfirst[sc[s]] = (int32_t)s;
}

__global__ void k_group_count(int64_t ng, int64_t n, const int32_t* __restrict__ gfirst, int32_t* __restrict__ gcount) {
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= ng) return;
    int32_t e = (g + 1 < ng) ? gfirst[g + 1] : (int32_t)n;
    gcount[g] = e - gfirst[g];
}

// Tight boxes: 16 lanes per group, lane j taking the group's particles
// j, j + 16, ... (min and max are exact in any order).
constexpr int kBoxLanes = 16;

__global__ __launch_bounds__(256) void k_group_bbox(int64_t ng, const int32_t* __restrict__ gfirst,
                                                    const int32_t* __restrict__ gcount, const double* __restrict__ px,
                                                    const double* __restrict__ py, const double* __restrict__ pz,
                                                    double* __restrict__ lo, double* __restrict__ hi) {
    const int64_t g = blockIdx.x * (int64_t)(256 / kBoxLanes) + threadIdx.x / kBoxLanes;
    const int j = threadIdx.x & (kBoxLanes - 1);
    double a[3], b[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a[k] = INFINITY;
        b[k] = -INFINITY;
    }
    if (g < ng) {
        const int32_t f = gfirst[g], cnt = gcount[g];
        for (int32_t q = j; q < cnt; q += kBoxLanes) {
            const double v[3] = {px[f + q], py[f + q], pz[f + q]};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                a[k] = v[k] < a[k] ? v[k] : a[k];
                b[k] = v[k] > b[k] ? v[k] : b[k];
            }
        }
    }
#pragma unroll
    for (int o = kBoxLanes / 2; o >= 1; o >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double u = __shfl_xor(a[k], o, kBoxLanes);
            const double w = __shfl_xor(b[k], o, kBoxLanes);
            a[k] = u < a[k] ? u : a[k];
            b[k] = w > b[k] ? w : b[k];
        }
    }
    if (g < ng && j == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[g * 3 + k] = a[k];
            hi[g * 3 + k] = b[k];
        }
    }
}

int64_t read_i32(const int32_t* d, hipStream_t st) {
    int32_t h = 0;
    SRF_HIP(hipMemcpyAsync(&h, d, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SRF_HIP(hipStreamSynchronize(st));
    return h;
}

}  // namespace

void build_cells_and_groups(Tree& t, int32_t* d_flag, hipStream_t st) {
    (void)d_flag;
    const int64_t n = t.n;
    const int B = 256;
    Bfs b;
    bfs_alloc(b, std::max<int64_t>(1024, n / 4 + 64), st);
    hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, st, n, b.level.get(), b.first.get(), b.count.get(),
                       b.parent.get(), b.prefix.get());
    SRF_HIP(hipGetLastError());
    std::vector<int64_t> lvl_off{0, 1};
    int64_t cur_begin = 0, cur_end = 1;
    int max_level = 0;
    for (int L = 0; L < kMaxLevel; ++L) {
        const int64_t m = cur_end - cur_begin;
        DevBuf<int32_t> bnd(m * 9, st), cnt(m + 1, st);
        hipLaunchKernelGGL(k_child_count, dim3(grid_for(m, 32, 1 << 30)), dim3(256), 0, st, cur_begin, m, L,
                           t.n_leaf, b.first.get(), b.count.get(), t.keys.get(), bnd.get(), cnt.get());
        SRF_HIP(hipGetLastError());
        exclusive_scan_i32(cnt.get(), m, true, st);
        const int64_t c = read_i32(cnt.get() + m, st);
        if (c == 0) {
            hipLaunchKernelGGL(k_leaf_fix, dim3(grid_for(m, B, 1 << 30)), dim3(B), 0, st, cur_begin, m,
                               b.child_begin.get(), b.child_cnt.get());
            SRF_HIP(hipGetLastError());
            break;
        }
        bfs_grow(b, cur_end, cur_end + c, st);
        hipLaunchKernelGGL(k_child_write, dim3(grid_for(m, B, 1 << 30)), dim3(B), 0, st, cur_begin, m, cur_end, L,
                           bnd.get(), cnt.get(), b.level.get(), b.first.get(), b.count.get(), b.parent.get(),
                           b.child_begin.get(), b.child_cnt.get(), b.prefix.get());
        SRF_HIP(hipGetLastError());
        cur_begin = cur_end;
        cur_end += c;
        lvl_off.push_back(cur_end);
        max_level = L + 1;
        if (max_level == kMaxLevel) {
            const int64_t mm = cur_end - cur_begin;
            hipLaunchKernelGGL(k_leaf_fix, dim3(grid_for(mm, B, 1 << 30)), dim3(B), 0, st, cur_begin, mm,
                               b.child_begin.get(), b.child_cnt.get());
            SRF_HIP(hipGetLastError());
        }
    }
    const int64_t nn = cur_end;
    t.n_nodes = nn;
    t.max_level = max_level;

    // moments, deepest level first
    DevBuf<double> M(nn, st), SX(nn, st), SY(nn, st), SZ(nn, st);
    for (int L = (int)lvl_off.size() - 2; L >= 0; --L) {
        const int64_t beg = lvl_off[L], m = lvl_off[L + 1] - lvl_off[L];
        hipLaunchKernelGGL(k_moments, dim3(grid_for(m, 256 / kMomLanes, 1 << 30)), dim3(256), 0, st, beg, m,
                           b.first.get(), b.count.get(), b.child_begin.get(), b.child_cnt.get(), t.px.get(),
                           t.py.get(), t.pz.get(), t.pm.get(), M.get(), SX.get(), SY.get(), SZ.get());
        SRF_HIP(hipGetLastError());
    }

    // preorder renumbering
    DevBuf<int32_t> cntf(n + 1, st), minlv(n + 1, st), bfs2pre(nn, st);
    fill_i32(cntf.get(), 0, n + 1, st);
    hipLaunchKernelGGL(k_pre_count, dim3(grid_for(nn, B, 1 << 30)), dim3(B), 0, st, nn, b.first.get(), b.level.get(),
                       b.parent.get(), b.child_cnt.get(), cntf.get(), minlv.get());
    SRF_HIP(hipGetLastError());
    exclusive_scan_i32(cntf.get(), n, true, st);  // cntf[n] = nn
    hipLaunchKernelGGL(k_pre_assign, dim3(grid_for(nn, B, 1 << 30)), dim3(B), 0, st, nn, b.first.get(),
                       b.level.get(), cntf.get(), minlv.get(), bfs2pre.get());
    SRF_HIP(hipGetLastError());
    t.geo.alloc(nn, st);
    t.range.alloc(nn, st);
    t.pack.alloc(nn, st);
    t.prefix.alloc(nn, st);
    t.nM.alloc(nn, st);
    t.nX.alloc(nn, st);
    t.nY.alloc(nn, st);
    t.nZ.alloc(nn, st);
    t.leaf_of.alloc(n, st);
    hipLaunchKernelGGL(k_pre_scatter, dim3(grid_for(nn, B, 1 << 30)), dim3(B), 0, st, nn, n, bfs2pre.get(),
                       b.level.get(), b.first.get(), b.count.get(), b.parent.get(), b.child_cnt.get(), b.prefix.get(),
                       cntf.get(), M.get(), SX.get(), SY.get(), SZ.get(), t.geo.get(), t.range.get(), t.pack.get(),
                       t.prefix.get(),
                       t.nM.get(), t.nX.get(), t.nY.get(), t.nZ.get(), t.leaf_of.get());
    SRF_HIP(hipGetLastError());

    // groups
    DevBuf<int32_t> mark(n + 1, st);
    fill_i32(mark.get(), 0, n + 1, st);
    hipLaunchKernelGGL(k_group_marks, dim3(grid_for(nn, B, 1 << 30)), dim3(B), 0, st, nn, t.n_group, t.geo.get(),
                       t.range.get(), mark.get());
    SRF_HIP(hipGetLastError());
    exclusive_scan_i32(mark.get(), n, true, st);
    const int64_t ng = read_i32(mark.get() + n, st);
    t.n_groups = ng;
    t.gfirst.alloc(ng, st);
    t.gcount.alloc(ng, st);
    t.glo.alloc(ng * 3, st);
    t.ghi.alloc(ng * 3, st);
    hipLaunchKernelGGL(k_group_write, dim3(grid_for(n, B, 1 << 30)), dim3(B), 0, st, n, mark.get(), t.gfirst.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_group_count, dim3(grid_for(ng, B, 1 << 30)), dim3(B), 0, st, ng, n, t.gfirst.get(),
                       t.gcount.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_group_bbox, dim3(grid_for(ng, 256 / kBoxLanes, 1 << 30)), dim3(256), 0, st, ng, t.gfirst.get(),
                       t.gcount.get(), t.px.get(), t.py.get(), t.pz.get(), t.glo.get(), t.ghi.get());
    SRF_HIP(hipGetLastError());
}

}  // namespace srf
