// Step a6: per-group interaction lists (Barnes' modified traversal with the
// cutoff pruning of the short-range part).
//
// Threads walk the preorder cell array without a stack: a cell that is
// pruned, accepted or a leaf is left through its skip link, any other cell
// is opened by stepping to the next preorder index (its first child).  A
// count pass sizes the lists, a scan places them, and a write pass emits
// one item per leaf or accepted cell in DFS order; an expansion pass then
// writes the entries (a leaf's particles ascending, cells in preorder) with
// one wave per group, so that the list memory is written in whole lines.
//
// Compiled with -ffp-contract=off: the decisions are the literal FP64
// expressions, evaluated in this order:
//   per axis t = |cen_c - cen_g|, t = min(t, 1 - t), e = max(0, t - (half + h_g))
//   d2 = (e_x e_x + e_y e_y) + e_z e_z
//   prune  iff d2(half = side/2) >= r_cut * r_cut
//   accept iff side * side < (theta * theta) * d2(half = 0)
// with cen_c the cell's geometric centre, or for the acceptance test of the
// centre-of-mass criterion its centre of mass.  A refitted tree measures
// each cell by the box [lo, hi] of its particles instead, every bound
// rounded outward to a multiple of 2^-(level + 10) (a cell whose bounds do
// not fit 16-bit offsets from its centre is never pruned or accepted):
//   cen_c = (lo + hi) * 0.5, half = (hi - lo) * 0.5 per axis,
//   per axis t = cen_c - cen_g, t = |t - rint(t)|, e = max(0, t - (half + h_g))
//   d2 as above; prune iff d2 >= r_cut * r_cut,
//   accept iff s * s < (theta * theta) * d2(half = 0, cen_c or the centre of mass),
// s the larger of the cell's dyadic side and the box's longest side
// (2 max(half)), so that a cell holding a member of the group is never
// accepted, however small its box.  For a fresh tree the walk first takes
// the two tests in FP32 with an error margin, and evaluates the FP64
// expressions only for the few cells whose FP32 values lie within the
// margin of a threshold (classify32 below): the decisions, and so the
// lists, are those of the FP64 expressions.
#include <type_traits>

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

// Decoded cell: exact centre and side.
struct Cell {
    double c[3], side, hs;
    int level, leaf;
    uint32_t count;
    int64_t skip;
};

// The cell of an 8-byte walk record, its coordinates found from those of
// the cell visited before (w): the new cell's parent is that cell or one of
// its ancestors, at level k.level - 1, whose coordinates are w's shifted
// down by the levels between; the cell's own low bits are `oct`.
struct WalkPos {
    uint32_t ix = 0, iy = 0, iz = 0;
    int level = -1;
};

__device__ __forceinline__ Cell decode_walk(const uint2 r, WalkPos& w) {
    Cell k;
    k.level = (int)(r.x & 31u);
    k.leaf = (int)((r.x >> 5) & 1u);
    const uint32_t oct = (r.x >> 6) & 7u;
    k.count = r.x >> 9;
    k.skip = (int64_t)r.y;
    const int sh = w.level + 1 - k.level;
    w.ix = ((w.ix >> sh) << 1) | (oct >> 2);
    w.iy = ((w.iy >> sh) << 1) | ((oct >> 1) & 1u);
    w.iz = ((w.iz >> sh) << 1) | (oct & 1u);
    w.level = k.level;
    return k;
}

// The exact centre and side of the cell last decoded into w.
__device__ __forceinline__ void cell_geometry(Cell& k, const WalkPos& w) {
    k.side = ldexp(1.0, -k.level);
    k.hs = k.side * 0.5;
    k.c[0] = ldexp((double)w.ix + 0.5, -k.level);
    k.c[1] = ldexp((double)w.iy + 0.5, -k.level);
    k.c[2] = ldexp((double)w.iz + 0.5, -k.level);
}

__device__ __forceinline__ Cell decode(const uint4 r) {
    Cell k;
    k.level = (int)(r.w & 31u);
    k.leaf = (int)((r.w >> 5) & 1u);
    k.count = r.w >> 6;
    k.skip = (int64_t)((r.x >> 21) | ((r.y >> 21) << 11) | ((r.z >> 21) << 22));
    k.side = ldexp(1.0, -k.level);
    k.hs = k.side * 0.5;
    k.c[0] = ldexp((double)(r.x & 0x1fffffu) + 0.5, -k.level);
    k.c[1] = ldexp((double)(r.y & 0x1fffffu) + 0.5, -k.level);
    k.c[2] = ldexp((double)(r.z & 0x1fffffu) + 0.5, -k.level);
    return k;
}

// 0: pruned, 1: accepted as a monopole, 2: leaf (expand), 3: open.  `mc`
// is the point the acceptance test measures to (the geometric centre, or
// the centre of mass with the centre-of-mass criterion).
__device__ __forceinline__ int classify(const Cell& k, const double* mc, const Frame& f, double rc2, double th2) {
    double ex = axis_gap(k.c[0], f.cg[0], k.hs + f.hg[0]);
    double ey = axis_gap(k.c[1], f.cg[1], k.hs + f.hg[1]);
    double ez = axis_gap(k.c[2], f.cg[2], k.hs + f.hg[2]);
    double D2 = (ex * ex + ey * ey) + ez * ez;
    if (D2 >= rc2) return 0;
    ex = axis_gap(mc[0], f.cg[0], f.hg[0]);
    ey = axis_gap(mc[1], f.cg[1], f.hg[1]);
    ez = axis_gap(mc[2], f.cg[2], f.hg[2]);
    double d2 = (ex * ex + ey * ey) + ez * ez;
    if (k.side * k.side < th2 * d2) return 1;
    return k.leaf ? 2 : 3;
}

// A first look in FP32 at the same two tests.  Every quantity before the
// squares is within 4e-7 of its exact value (the centres are exact in FP32,
// the group's centre and half sizes are rounded once, and each of the four
// operations per axis rounds a value below 1), so a squared distance D2 is
// within 1.4e-6 sqrt(D2) + 2.4e-7 D2 + 1e-12 of its exact value; FP64 is
// within 1e-15.  A test is decided here only when the FP32 value clears its
// threshold X by more than b(X) = 2.5e-6 sqrt(X) + 2e-6 X + 1e-12, which
// exceeds both errors together, so that the FP64 expressions would decide
// the same way; otherwise (-1) they are evaluated.
struct Frame32 {
    float cg[3], hg[3];
};

__device__ __forceinline__ float axis_gap32(float cen, float cg, float half) {
    float t = fabsf(cen - cg);
    const float t2 = 1.0f - t;
    t = t2 < t ? t2 : t;
    const float r = t - half;
    return r > 0.0f ? r : 0.0f;
}

// rc_hi / rc_lo: r_cut^2 +- b(r_cut^2); inv_th: 1 / theta.
__device__ __forceinline__ int classify32(int level, int leaf, const float* c, const float* mc, const Frame32& f,
                                          float rc_hi, float rc_lo, float inv_th) {
    const float side = __int_as_float((127 - level) << 23);   // 2^-level, exact
    const float hs = side * 0.5f;
    float ex = axis_gap32(c[0], f.cg[0], hs + f.hg[0]);
    float ey = axis_gap32(c[1], f.cg[1], hs + f.hg[1]);
    float ez = axis_gap32(c[2], f.cg[2], hs + f.hg[2]);
    const float D2 = (ex * ex + ey * ey) + ez * ez;
    if (D2 >= rc_hi) return 0;
    if (!(D2 < rc_lo)) return -1;
    ex = axis_gap32(mc[0], f.cg[0], f.hg[0]);
    ey = axis_gap32(mc[1], f.cg[1], f.hg[1]);
    ez = axis_gap32(mc[2], f.cg[2], f.hg[2]);
    const float d2 = (ex * ex + ey * ey) + ez * ez;
    const float sx = side * inv_th, X = sx * sx;   // accept iff d2 > side^2 / theta^2
    const float b = 2.5e-6f * sx + 2e-6f * X + 1e-12f;
    if (d2 > X + b) return 1;
    if (!(d2 < X - b)) return -1;
    return leaf ? 2 : 3;
}

__device__ __forceinline__ double refit_axis_gap(double cen, double cg, double half) {
    double t = cen - cg;
    t = fabs(t - rint(t));
    double r = t - half;
    return r > 0.0 ? r : 0.0;
}

// The rounded box of a refitted cell: bound K q with K the stored offset
// plus the centre's multiple ic * 1024 + 512 (exact in FP64).
__device__ __forceinline__ void refit_box(const RefitCell& r, const Cell& k, double* bl, double* bh) {
    const uint32_t ic[3] = {r.pk.x & 0x1fffffu, r.pk.y & 0x1fffffu, r.pk.z & 0x1fffffu};
    const int e = k.level + kRefitShift;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t kc = (int64_t)ic[a] * (1 << kRefitShift) + (1 << (kRefitShift - 1));
        const int32_t lo = (int32_t)(int16_t)(r.b[a] & 0xffff), hi = r.b[a] >> 16;
        bl[a] = ldexp((double)(kc + lo), -e);
        bh[a] = ldexp((double)(kc + hi), -e);
    }
}

// The same classification for a cell of a refitted tree with box [bl, bh].
__device__ __forceinline__ int classify_refit(const Cell& k, const double* bl, const double* bh, const double* mc,
                                              bool com, const Frame& f, double rc2, double th2) {
    double cen[3], half[3], hmax = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cen[a] = (bl[a] + bh[a]) * 0.5;
        half[a] = (bh[a] - bl[a]) * 0.5;
        hmax = half[a] > hmax ? half[a] : hmax;
    }
    double side = hmax + hmax;
    side = k.side > side ? k.side : side;
    double ex = refit_axis_gap(cen[0], f.cg[0], half[0] + f.hg[0]);
    double ey = refit_axis_gap(cen[1], f.cg[1], half[1] + f.hg[1]);
    double ez = refit_axis_gap(cen[2], f.cg[2], half[2] + f.hg[2]);
    double D2 = (ex * ex + ey * ey) + ez * ez;
    if (D2 >= rc2) return 0;
    const double* m = com ? mc : cen;
    ex = refit_axis_gap(m[0], f.cg[0], 0.0 + f.hg[0]);
    ey = refit_axis_gap(m[1], f.cg[1], 0.0 + f.hg[1]);
    ez = refit_axis_gap(m[2], f.cg[2], 0.0 + f.hg[2]);
    double d2 = (ex * ex + ey * ey) + ez * ez;
    if (side * side < th2 * d2) return 1;
    return k.leaf ? 2 : 3;
}

// Items of one group pass through a 16-slot LDS buffer of the thread and go
// to memory as aligned 64-byte chunks (the partial chunks at the two ends of
// a group's items are written item by item), so that the item array is
// written in whole lines rather than by scattered 4-byte stores.
constexpr int kWc = 16;          // items per chunk
constexpr int kWcStride = 17;    // LDS slots per thread (padding against bank conflicts)

struct ItemWriter {
    int32_t* buf;      // this thread's LDS slots
    int32_t* dst;      // the item array
    int64_t start;     // index of the group's first item
    int64_t pos;       // index of the next item
    int64_t end;       // capacity limit: items at or past `end` are counted, not stored
    __device__ __forceinline__ void put(int32_t v) {
        if (pos < end) buf[pos & (kWc - 1)] = v;
        ++pos;
        if ((pos & (kWc - 1)) == 0 && pos <= end) {
            const int64_t c0 = pos - kWc;
            if (c0 >= start) {
                int4* d = reinterpret_cast<int4*>(dst + c0);
#pragma unroll
                for (int k = 0; k < kWc / 4; ++k) d[k] = make_int4(buf[4 * k], buf[4 * k + 1], buf[4 * k + 2], buf[4 * k + 3]);
            } else {
                for (int64_t k = start; k < pos; ++k) dst[k] = buf[k & (kWc - 1)];
            }
        }
    }
    __device__ __forceinline__ void finish() {
        if (pos > end) return;
        int64_t k = pos & ~(int64_t)(kWc - 1);
        if (k < start) k = start;
        for (; k < pos; ++k) dst[k] = buf[k & (kWc - 1)];
    }
};

// One thread walks the cell array once for G consecutive groups.  A cell
// is visited while at least one of them opened its parent; mask[L] (G bits
// per level, packed in one 64-bit word) holds the groups that opened the
// visited cell's parent at level L - 1.
//
// The counting walk (WRITE = false) sizes each group's list and also stores
// its items into a slot of kSlot items per group (items past the slot are
// counted in totals[3], and the lists are then rebuilt with WRITE = true:
// a second walk that stores the items of every group compactly at ioff).
constexpr int64_t kSlot = 2048;
constexpr int kListThreads = 64;   // one wave per block (128 and 256 measured slower)

template <int G, bool WRITE, bool COM, bool REFIT>
__global__ __launch_bounds__(kListThreads) void k_lists(int64_t ng, const double* __restrict__ glo,
                                               const double* __restrict__ ghi, const int32_t* __restrict__ gcount,
                                               const uint2* __restrict__ pack, const NodeRange* __restrict__ rng,
                                               const double* __restrict__ nX, const double* __restrict__ nY,
                                               const double* __restrict__ nZ,
                                               const RefitCell* __restrict__ rpack, int64_t nn, double rc2, double th2, int64_t* __restrict__ cnt,
                                               int64_t* __restrict__ icnt, unsigned long long* __restrict__ totals,
                                               const int64_t* __restrict__ ioff, int32_t* __restrict__ items) {
    static_assert(G * kLevels <= 64, "level masks must fit one word");
    const int64_t t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int64_t g0 = t * G;
    __shared__ int32_t wbuf[kListThreads * G * kWcStride];
    Frame f[G];
    int64_t np[G], nc[G], w[G];
    ItemWriter out[G];
    uint64_t valid = 0;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        np[q] = nc[q] = w[q] = 0;
        const int64_t g = g0 + q < ng ? g0 + q : ng - 1;
        f[q] = group_frame(glo, ghi, g);
        if (g0 + q < ng) valid |= 1ull << q;
        out[q].buf = wbuf + (threadIdx.x * G + q) * kWcStride;
        out[q].dst = items;
        out[q].start = out[q].pos = WRITE ? ioff[g] : g * kSlot;
        out[q].end = WRITE ? INT64_MAX : g * kSlot + kSlot;
    }
    Frame32 f32[G];
#pragma unroll
    for (int q = 0; q < G; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            f32[q].cg[a] = (float)f[q].cg[a];
            f32[q].hg[a] = (float)f[q].hg[a];
        }
    const float rc2f = (float)rc2;
    const float bp = 2.5e-6f * sqrtf(rc2f) + 2e-6f * rc2f + 1e-12f;
    const float rc_hi = rc2f + bp, rc_lo = rc2f - bp;
    const float inv_th = th2 > 0.0 ? (float)(1.0 / sqrt(th2)) : INFINITY;
    const uint64_t full = (1ull << G) - 1ull;
    uint64_t masks = valid;  // level 0
    int64_t i = valid ? 0 : nn;
    WalkPos wpos;
    while (i < nn) {
        RefitCell rc;
        if (REFIT) rc = rpack[i];
        Cell k = REFIT ? decode(rc.pk) : decode_walk(pack[i], wpos);
        const uint64_t act = (masks >> (k.level * G)) & full;
        uint64_t open = 0;
        if (act) {
            float c32[3] = {0.0f, 0.0f, 0.0f}, mc32[3] = {0.0f, 0.0f, 0.0f};
            double com[3] = {0.0, 0.0, 0.0};
            if (!REFIT) {
                const float side32 = __int_as_float((127 - k.level) << 23);
                const float hs32 = side32 * 0.5f;
                // (i + 1/2) 2^-level: exact in FP32 (i < 2^21)
                c32[0] = __fmaf_rn((float)wpos.ix, side32, hs32);
                c32[1] = __fmaf_rn((float)wpos.iy, side32, hs32);
                c32[2] = __fmaf_rn((float)wpos.iz, side32, hs32);
                mc32[0] = c32[0];
                mc32[1] = c32[1];
                mc32[2] = c32[2];
            }
            if (COM) {
                com[0] = nX[i];
                com[1] = nY[i];
                com[2] = nZ[i];
                mc32[0] = (float)com[0];
                mc32[1] = (float)com[1];
                mc32[2] = (float)com[2];
            }
            bool geom = REFIT;   // FP64 geometry computed (a refitted cell's comes with its record)
            double mcen[3] = {0.0, 0.0, 0.0};
            if (REFIT) {
                mcen[0] = COM ? com[0] : k.c[0];
                mcen[1] = COM ? com[1] : k.c[1];
                mcen[2] = COM ? com[2] : k.c[2];
            }
            double bl[3] = {0, 0, 0}, bh[3] = {0, 0, 0};
            bool bounded = true;
            if (REFIT) {
                bounded = rc.b[3] & 1;
                refit_box(rc, k, bl, bh);
            }
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (!((act >> q) & 1ull)) continue;
                int cls;
                if (REFIT) {
                    cls = bounded ? classify_refit(k, bl, bh, mcen, COM, f[q], rc2, th2) : (k.leaf ? 2 : 3);
                } else {
                    cls = classify32(k.level, k.leaf, c32, mc32, f32[q], rc_hi, rc_lo, inv_th);
                    if (cls < 0) {
                        if (!geom) {
                            cell_geometry(k, wpos);
                            mcen[0] = COM ? com[0] : k.c[0];
                            mcen[1] = COM ? com[1] : k.c[1];
                            mcen[2] = COM ? com[2] : k.c[2];
                            geom = true;
                        }
                        cls = classify(k, mcen, f[q], rc2, th2);
                    }
                }
                if (cls == 3) {
                    open |= 1ull << q;
                } else if (cls == 1) {
                    out[q].put(-(int32_t)i - 1);
                    if (!WRITE) ++nc[q];
                } else if (cls == 2) {
                    out[q].put((int32_t)i);
                    if (!WRITE) {
                        uint32_t m = k.count;
                        if (m == (REFIT ? kPackCountMax : kWalkCountMax)) m = (uint32_t)rng[i].count;
                        np[q] += m;
                        ++w[q];
                    }
                }
            }
        }
        if (open) {
            const int sh = (k.level + 1) * G;
            masks = (masks & ~(full << sh)) | (open << sh);
            ++i;
        } else {
            i = k.skip;
        }
    }
#pragma unroll
    for (int q = 0; q < G; ++q)
        if ((valid >> q) & 1ull) out[q].finish();
    if (WRITE) return;
    unsigned long long a = 0, b = 0, c = 0, d = 0;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        if (!((valid >> q) & 1ull)) continue;
        cnt[g0 + q] = np[q] + nc[q];
        icnt[g0 + q] = w[q] + nc[q];   // leaves + accepted cells
        a += (unsigned long long)np[q];
        b += (unsigned long long)nc[q];
        c += (unsigned long long)gcount[g0 + q] * (unsigned long long)(np[q] + nc[q]);
        d += (w[q] + nc[q] > kSlot) ? 1ull : 0ull;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
        d += __shfl_xor(d, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&totals[0], a);
        atomicAdd(&totals[1], b);
        atomicAdd(&totals[2], c);
        if (d) atomicAdd(&totals[3], d);
    }
}

// Expansion: one wave per group turns its items into entries.  A leaf item
// stands for its particles first..first+count-1, a cell item for itself.
// Items are taken kExpandItems at a time: each lane loads four of them, the
// next batch's four while it places these, and the four items' ranges (all
// of a batch's range loads in flight together), a scan of the item sizes
// places each item, and the entries are written
// either through an LDS buffer (each lane writes its own items' entries,
// then the wave copies the buffer out, 64 consecutive entries per store) or,
// when the batch's entries exceed the buffer, directly, lane k writing
// entries k, k + 64, ... and finding its item by binary search over the
// scan.
// Items of group g: icnt[g] of them from g * slot when slot > 0, else
// [ioff[g], ioff[g + 1]).
constexpr int kExpandBuf = 1024;
constexpr int kExpandPer = 4;                   // items per lane per batch
constexpr int kExpandItems = 64 * kExpandPer;   // items per batch

__global__ __launch_bounds__(64) void k_expand(int64_t ng, int64_t slot, const int64_t* __restrict__ icnt,
                                               const int64_t* __restrict__ ioff, const int32_t* __restrict__ items,
                                               const NodeRange* __restrict__ rng, const int64_t* __restrict__ off,
                                               int32_t* __restrict__ ent) {
    __shared__ int32_t s_end[kExpandItems], s_first[kExpandItems];
    __shared__ int32_t s_ent[kExpandBuf];
    const int64_t g = xcd_block(blockIdx.x, gridDim.x);
    if (g >= ng) return;
    const int lane = threadIdx.x;
    const int64_t i0 = slot > 0 ? g * slot : ioff[g];
    const int64_t i1 = slot > 0 ? i0 + icnt[g] : ioff[g + 1];
    int32_t* dst = ent + off[g];
    // item q = 64 k + lane of the batch at c0
    int32_t v[kExpandPer];
#pragma unroll
    for (int k = 0; k < kExpandPer; ++k) {
        const int64_t ii = i0 + 64 * k + lane;
        v[k] = ii < i1 ? items[ii] : INT32_MIN;
    }
    for (int64_t c0 = i0; c0 < i1; c0 += kExpandItems) {
        // every lane loads a range (a cell item or an empty place that of
        // cell 0, unused), so that no branch separates the batch's loads
        int32_t rf[kExpandPer], rc[kExpandPer], vn[kExpandPer], first[kExpandPer], n[kExpandPer];
#pragma unroll
        for (int k = 0; k < kExpandPer; ++k) {
            const NodeRange& r = rng[v[k] >= 0 ? v[k] : 0];
            rf[k] = r.first;
            rc[k] = r.count;
        }
#pragma unroll
        for (int k = 0; k < kExpandPer; ++k) {
            const int64_t ii = c0 + kExpandItems + 64 * k + lane;
            vn[k] = ii < i1 ? items[ii] : INT32_MIN;
        }
#pragma unroll
        for (int k = 0; k < kExpandPer; ++k) {
            first[k] = v[k] >= 0 ? rf[k] : v[k];
            n[k] = v[k] >= 0 ? rc[k] : (v[k] == INT32_MIN ? 0 : 1);
        }
        uint64_t leafmask[kExpandPer];
        int carry = 0;
        int incl[kExpandPer];
#pragma unroll
        for (int k = 0; k < kExpandPer; ++k) {
            int x = n[k];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int u = __shfl_up(x, o, 64);
                if (lane >= o) x += u;
            }
            incl[k] = x + carry;
            carry += __shfl(x, 63, 64);
            leafmask[k] = __ballot(v[k] >= 0 && n[k] > 0);
        }
        const int total = carry;
        if (total <= kExpandBuf) {
            // a leaf's entries are first, first + 1, ...; a cell's only
            // entry is its code
#pragma unroll
            for (int k = 0; k < kExpandPer; ++k) {
                const int b = incl[k] - n[k];
                if (v[k] >= 0) {
                    for (int q = 0; q < n[k]; ++q) s_ent[b + q] = first[k] + q;
                } else if (n[k] > 0) {
                    s_ent[b] = first[k];
                }
            }
            __syncthreads();
            for (int k = lane; k < total; k += 64) dst[k] = s_ent[k];
            __syncthreads();
        } else {
#pragma unroll
            for (int k = 0; k < kExpandPer; ++k) {
                s_end[64 * k + lane] = incl[k];
                s_first[64 * k + lane] = v[k] >= 0 ? first[k] - (incl[k] - n[k]) : first[k];
            }
            __syncthreads();
            for (int e = lane; e < total; e += 64) {
                // first item whose end exceeds e
                int lo = 0;
#pragma unroll
                for (int step = kExpandItems / 2; step >= 1; step >>= 1)
                    if (s_end[lo + step - 1] <= e) lo += step;
                const int32_t f = s_first[lo];
                dst[e] = ((leafmask[lo >> 6] >> (lo & 63)) & 1ull) ? f + e : f;
            }
            __syncthreads();
        }
        dst += total;
#pragma unroll
        for (int k = 0; k < kExpandPer; ++k) v[k] = vn[k];
    }
}

constexpr int kGroupsPerThread = 1;

}  // namespace

void build_lists(const Tree& t, Lists& l, hipStream_t st) {
    const int64_t ng = t.n_groups;
    const double rc2 = l.r_cut * l.r_cut;
    const double th2 = l.theta * l.theta;
    l.n_groups = ng;
    l.off.alloc(ng + 1, st);
    DevBuf<int64_t> icnt(ng + 1, st);
    DevBuf<int32_t> slots(ng * kSlot > 0 ? ng * kSlot : 1, st);
    DevBuf<unsigned long long> totals(4, st);
    fill_u64(totals.get(), 0ull, 4, st);
    const int B = kListThreads;
    constexpr int G = kGroupsPerThread;
    const int64_t nthreads = (ng + G - 1) / G;
    const dim3 grid(grid_for(nthreads, B, 1 << 30)), block(B);
    const bool com = l.mac == SRF_MAC_COM;
    // the walk for this tree: geometric or refitted cells, either criterion
    auto walk = [&](auto kernel, int64_t* cnt, int64_t* ic, unsigned long long* tot, const int64_t* ioff,
                    int32_t* out) {
        hipLaunchKernelGGL(kernel, grid, block, 0, st, ng, t.glo.get(), t.ghi.get(), t.gcount.get(), t.pack.get(),
                           t.range.get(), t.nX.get(), t.nY.get(), t.nZ.get(), t.rpack.get(), t.n_nodes,
                           rc2, th2, cnt, ic, tot, ioff, out);
    };
    auto walk_all = [&](auto write, int64_t* cnt, int64_t* ic, unsigned long long* tot, const int64_t* ioff,
                        int32_t* out) {
        constexpr bool W = decltype(write)::value;
        if (t.refit) {
            if (com) walk(k_lists<G, W, true, true>, cnt, ic, tot, ioff, out);
            else walk(k_lists<G, W, false, true>, cnt, ic, tot, ioff, out);
        } else {
            if (com) walk(k_lists<G, W, true, false>, cnt, ic, tot, ioff, out);
            else walk(k_lists<G, W, false, false>, cnt, ic, tot, ioff, out);
        }
    };
    walk_all(std::false_type{}, l.off.get(), icnt.get(), totals.get(), (const int64_t*)nullptr, slots.get());
    SRF_HIP(hipGetLastError());
    exclusive_scan_i64(l.off.get(), ng, true, st);
    unsigned long long h[4];
    SRF_HIP(hipMemcpyAsync(h, totals.get(), 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SRF_HIP(hipStreamSynchronize(st));
    l.n_particle_entries = (int64_t)h[0];
    l.n_node_entries = (int64_t)h[1];
    l.n_entries = (int64_t)(h[0] + h[1]);
    l.interactions = (int64_t)h[2];
    l.ent.alloc(l.n_entries > 0 ? l.n_entries : 1, st);
    if (ng == 0) return;
    if (h[3] == 0) {
        // every group's items fit its slot
        hipLaunchKernelGGL(k_expand, dim3((unsigned)ng), dim3(64), 0, st, ng, kSlot, icnt.get(),
                           (const int64_t*)nullptr, slots.get(), t.range.get(), l.off.get(), l.ent.get());
        SRF_HIP(hipGetLastError());
        return;
    }
    // some group has more items than a slot holds: walk again and store
    // every group's items compactly
    slots.reset();
    exclusive_scan_i64(icnt.get(), ng, true, st);
    int64_t n_items = 0;
    SRF_HIP(hipMemcpyAsync(&n_items, icnt.get() + ng, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    SRF_HIP(hipStreamSynchronize(st));
    DevBuf<int32_t> items(n_items > 0 ? n_items : 1, st);
    walk_all(std::true_type{}, (int64_t*)nullptr, (int64_t*)nullptr, (unsigned long long*)nullptr,
             (const int64_t*)icnt.get(), items.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_expand, dim3((unsigned)ng), dim3(64), 0, st, ng, (int64_t)0, (const int64_t*)nullptr,
                       icnt.get(), items.get(), t.range.get(), l.off.get(), l.ent.get());
    SRF_HIP(hipGetLastError());
}

}  // namespace srf
