// Steps a3-a5 with one host synchronisation: the octree, its monopole
// moments, the DFS preorder with subtree "skip" links, the particle groups
// and their bounding boxes, all derived from the sorted Morton keys.
//
// Let delta(s) be the number of leading 3-bit digits that keys s-1 and s
// share (-1 for s = 0).  The cell of level L holding particle s starts at s
// iff delta(s) < L, and ends before the next index e with delta(e) < L.  It
// holds at least W particles iff some run of W consecutive particles that
// contains s lies inside it, i.e. iff delta >= L over that run's interior.
// So the deepest level whose cell holding s has more than k particles is
//   lambda_k(s) = max over runs [t, t + k] containing s of min delta(t+1 .. t+k)
// (-1 if there is no such run), a max of mins over runs of at most 65
// particles, taken per particle from an LDS tile.  From it:
//   - s lies in the leaf of level leaf(s) = min(21, max(1, lambda_{n_leaf}(s) + 1))
//     (a cell is split iff it holds more than n_leaf particles; the root
//     always);
//   - the cells starting at s are the levels delta(s)+1 .. leaf(s), a chain
//     in which each is the first child of the one before: their preorder
//     numbers are start(s) + L - delta(s) - 1, start the exclusive scan of
//     the chain lengths, so the whole preorder follows from one scan;
//   - s lies in the group candidate of level max(1, lambda_{n_group}(s) + 1)
//     (lambda = 21: a level-21 cell with more than n_group particles, cut
//     into chunks of n_group); whether a candidate starts a group follows
//     from its left siblings, found by 64-lane scans of delta in LDS.
// Each level's cells also get consecutive slots ordered by first particle
// (per-block counts, scanned per level), so that a cell's children are one
// contiguous run of the next level's slots; counts, moments and skip links
// then follow bottom-up, one launch per level, sized from the level totals
// read at the one synchronisation.
//
// Compiled with -ffp-contract=off: the group boxes feed the list decisions,
// which must be the literal FP64 expressions.
#include <string>

#include "common.h"

namespace srf {
namespace {

constexpr int kLvThreads = 256;
constexpr int kLvTile = 1024;                      // particles per block
constexpr int kPer = kLvTile / kLvThreads;
constexpr int kHalo = 64;                          // runs hold at most 65 particles
constexpr int kLvSpan = kLvTile + 2 * kHalo;       // deltas of the range tables
constexpr int kLvRuns = kLvTile + kHalo;           // run starts
constexpr int kLog = 7;                            // range tables for lengths 1..64
constexpr int kLeft = 512;                         // left reach of the sibling scans (7 siblings of <= 64, + 64)
constexpr int kScanSpan = kLeft + kLvTile + kHalo; // deltas of the sibling scans

__device__ __forceinline__ int shared_digits(uint64_t a, uint64_t b) {
    const uint64_t x = a ^ b;   // keys use the low 63 bits
    return x ? (__clzll(x) - 1) / 3 : kMaxLevel;
}

__device__ __forceinline__ int floor_log2(int v) { return 31 - __clz(v); }

// First index in [lo, s] whose key equals keys[s] (sorted keys).
__device__ __forceinline__ int64_t first_equal(const uint64_t* __restrict__ keys, int64_t lo, int64_t s) {
    const uint64_t k = keys[s];
    int64_t hi = s;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Per particle: delta, leaf level, the chain length of the cells starting
// there and the group-start mark; per block and level the number of cells
// (blk[L * nblocks + block]), and per block the sums of the chain lengths
// and of the marks (rows kLevels and kLevels + 1 of blk).
//
// Group starts.  A candidate (level >= 1, at most n_group particles, parent
// the root or holding more than n_group) starts a group under the root, and
// under any other parent unless the greedy run of the candidate siblings
// before it (octant order, closed by a sibling with more than n_group
// particles or by an overflow) takes it in.  Candidates under a parent of
// level >= 1 are handled one at a time by the whole wave: the candidate's end
// and its left siblings' starts are each the nearest index, among the 64
// after (before) a position, with delta below the candidate's level; a
// sibling whose start is further away holds more than n_group particles and
// closes the run.
__global__ __launch_bounds__(kLvThreads) void k_levels(int64_t n, const uint64_t* __restrict__ keys, int n_leaf,
                                                       int n_group, int64_t nblocks, int8_t* __restrict__ delta,
                                                       int8_t* __restrict__ leaflv, int32_t* __restrict__ chain,
                                                       int32_t* __restrict__ mark, int32_t* __restrict__ blk) {
    __shared__ int8_t mn[kLog][kLvSpan];   // mn[k][j] = min delta over [j, j + 2^k)
    __shared__ int8_t mx[kLog][kLvRuns];   // mx[k][j] = max run minimum over run starts [j, j + 2^k)
    __shared__ int8_t dl[kScanSpan];       // delta of global index b0 - kLeft + j
    __shared__ unsigned lh[kLevels + 2];   // cells per level; the tile's chain and mark sums
    const int64_t b0 = blockIdx.x * (int64_t)kLvTile;
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < kLevels + 2) lh[tid] = 0;
    for (int j = tid; j < kScanSpan; j += kLvThreads) {
        const int64_t i = b0 - kLeft + j;
        int d = -1;
        if (i >= 1 && i < n) d = shared_digits(keys[i - 1], keys[i]);
        dl[j] = (int8_t)d;
    }
    __syncthreads();
    // range table of minima over [b0 - kHalo, b0 + kLvTile + kHalo)
    for (int j = tid; j < kLvSpan; j += kLvThreads) mn[0][j] = dl[j + kLeft - kHalo];
    __syncthreads();
    for (int k = 1; k < kLog; ++k) {
        const int h = 1 << (k - 1);
        for (int j = tid; j < kLvSpan; j += kLvThreads) {
            // entries whose range runs past the span are never queried
            const int a = mn[k - 1][j], b = j + h < kLvSpan ? mn[k - 1][j + h] : a;
            mn[k][j] = (int8_t)(a < b ? a : b);
        }
        __syncthreads();
    }
    int lam[2][kPer];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const int W = (w == 0 ? n_leaf : n_group) + 1;   // run length, 2..65
        const int kq = floor_log2(W - 1);
        // minimum of delta over the interior of the run starting at each t
        for (int j = tid; j < kLvRuns; j += kLvThreads) {
            const int64_t t = b0 - kHalo + j;
            int v = -1;
            if (t >= 0 && t + W - 1 <= n - 1) {
                const int a = mn[kq][j + 1], b = mn[kq][j + W - (1 << kq)];
                v = a < b ? a : b;
            }
            mx[0][j] = (int8_t)v;
        }
        __syncthreads();
        for (int k = 1; k < kLog; ++k) {
            const int h = 1 << (k - 1);
            for (int j = tid; j < kLvRuns; j += kLvThreads) {
                const int a = mx[k - 1][j], b = j + h < kLvRuns ? mx[k - 1][j + h] : a;
                mx[k][j] = (int8_t)(a > b ? a : b);
            }
            __syncthreads();
        }
        // maximum over the runs [s - W + 1, s] that contain s
        const int kr = floor_log2(W);
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int js = kHalo + tid + q * kLvThreads;
            const int a = mx[kr][js - W + 1], b = mx[kr][js - (1 << kr) + 1];
            lam[w][q] = a > b ? a : b;
        }
        __syncthreads();
    }
    int32_t csum = 0, msum = 0;   // this thread's chain lengths and group marks
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t s = b0 + tid + q * kLvThreads;   // a wave holds 64 consecutive particles
        const bool on = s < n;
        const int js = kLeft + tid + q * kLvThreads;  // index of s in dl
        const int d = dl[js];
        int ll = lam[0][q] + 1;
        ll = ll < 1 ? 1 : (ll > kMaxLevel ? kMaxLevel : ll);
        const int lg = lam[1][q];
        const int kap = lg + 1 > 1 ? lg + 1 : 1;
        int m = 0;
        bool walk = false;
        if (on) {
            delta[s] = (int8_t)d;
            leaflv[s] = (int8_t)ll;
            chain[s] = ll > d ? ll - d : 0;
            csum += ll > d ? ll - d : 0;
            for (int L = d + 1; L <= ll; ++L) atomicAdd(&lh[L], 1u);
            if (lg >= kMaxLevel) {
                m = ((s - first_equal(keys, 0, s)) % n_group) == 0;   // chunks of a level-21 cell
            } else if (d < kap) {
                if (kap == 1) m = 1;
                else walk = true;
            }
        }
        // candidates under a parent of level >= 1, one per wave iteration
        uint64_t todo = __ballot(walk);
        while (todo) {
            const int src = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int cs = __shfl(js, src, 64);
            const int ck = __shfl(kap, src, 64);
            const int64_t cg = __shfl(s, src, 64);
            // the candidate's end: the first delta below its level among the
            // next 64 (it holds at most n_group, so the end is among them)
            const int de = cg + 1 + lane < n ? dl[cs + 1 + lane] : -1;
            const uint64_t eb = __ballot(de < ck);
            const int64_t own = __ffsll((unsigned long long)eb);
            // left siblings back to the parent's start or a closing sibling;
            // they span at most 7 x 64 particles, inside the left reach
            int64_t cnt[7];
            int ns = 0;
            int pos = cs;
            while (ns < 7 && dl[pos] >= ck - 1) {   // pos is not the parent's first index
                const int jb = pos - 1 - lane;
                const int db = jb >= 0 ? dl[jb] : -1;
                const uint64_t bb = __ballot(db < ck);
                if (!bb) break;   // no start within 64: the sibling holds more than n_group
                const int c = __ffsll((unsigned long long)bb);
                if (c > n_group) break;
                cnt[ns++] = c;
                pos -= c;
            }
            int64_t run = 0;
            bool open = false;
            for (int k = ns - 1; k >= 0; --k) {
                if (open && run + cnt[k] <= n_group) {
                    run += cnt[k];
                } else {
                    run = cnt[k];
                    open = true;
                }
            }
            if (lane == src) m = !(open && run + own <= n_group);
        }
        if (on) mark[s] = m;
        msum += on ? m : 0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        csum += __shfl_xor(csum, o, 64);
        msum += __shfl_xor(msum, o, 64);
    }
    if (lane == 0) {
        atomicAdd(&lh[kLevels], (unsigned)csum);
        atomicAdd(&lh[kLevels + 1], (unsigned)msum);
    }
    __syncthreads();
    if (tid < kLevels + 2) blk[(int64_t)tid * nblocks + blockIdx.x] = (int32_t)lh[tid];
}

// In place, over the tiles of k_levels: the exclusive scans of the chain
// lengths (the preorder number of each chain's first cell) and of the group
// marks (the group number of each group start), each tile starting from its
// scanned sum (rows kLevels and kLevels + 1 of blk); entry n of each gets
// the total.  Thread t takes the tile's entries 4t .. 4t + 3.
__global__ __launch_bounds__(kLvThreads) void k_scan_tiles(int64_t n, int64_t nblocks, int32_t* __restrict__ chain,
                                                           int32_t* __restrict__ mark,
                                                           const int32_t* __restrict__ blk,
                                                           const int32_t* __restrict__ tot) {
    static_assert(kPer == 4, "four entries per thread");
    __shared__ int32_t wsum[kLvThreads / 64][2];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t s0 = blockIdx.x * (int64_t)kLvTile + kPer * tid;
    int32_t c[kPer], m[kPer];
    if (s0 + kPer <= n) {
        const int4 cv = *reinterpret_cast<const int4*>(chain + s0);
        const int4 mv = *reinterpret_cast<const int4*>(mark + s0);
        c[0] = cv.x, c[1] = cv.y, c[2] = cv.z, c[3] = cv.w;
        m[0] = mv.x, m[1] = mv.y, m[2] = mv.z, m[3] = mv.w;
    } else {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            c[k] = s0 + k < n ? chain[s0 + k] : 0;
            m[k] = s0 + k < n ? mark[s0 + k] : 0;
        }
    }
    const int32_t cs = c[0] + c[1] + c[2] + c[3], ms = m[0] + m[1] + m[2] + m[3];
    int32_t ci = cs, mi = ms;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t u = __shfl_up(ci, o, 64), v = __shfl_up(mi, o, 64);
        if (lane >= o) {
            ci += u;
            mi += v;
        }
    }
    if (lane == 63) {
        wsum[wid][0] = ci;
        wsum[wid][1] = mi;
    }
    __syncthreads();
    int32_t co = blk[(int64_t)kLevels * nblocks + blockIdx.x] + ci - cs;
    int32_t mo = blk[(int64_t)(kLevels + 1) * nblocks + blockIdx.x] + mi - ms;
#pragma unroll
    for (int w = 0; w < kLvThreads / 64; ++w) {
        if (w < wid) {
            co += wsum[w][0];
            mo += wsum[w][1];
        }
    }
    int32_t cx[kPer], mx[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        cx[k] = co;
        mx[k] = mo;
        co += c[k];
        mo += m[k];
    }
    if (s0 + kPer <= n) {
        *reinterpret_cast<int4*>(chain + s0) = make_int4(cx[0], cx[1], cx[2], cx[3]);
        *reinterpret_cast<int4*>(mark + s0) = make_int4(mx[0], mx[1], mx[2], mx[3]);
    } else {
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (s0 + k < n) {
                chain[s0 + k] = cx[k];
                mark[s0 + k] = mx[k];
            }
        }
    }
    if (blockIdx.x == 0 && tid == 0) {
        chain[n] = tot[kLevels];
        mark[n] = tot[kLevels + 1];
    }
}

// Exclusive scan of one level's per-block cell counts (block = level), in
// place; the level's total goes to tot.  Rows kLevels and kLevels + 1 (the
// tiles' chain and mark sums) are scanned the same way.
__global__ __launch_bounds__(256) void k_level_scan(int64_t nblocks, int32_t* __restrict__ blk,
                                                    int32_t* __restrict__ tot) {
    constexpr int kItems = 4;
    __shared__ int32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int32_t* row = blk + (int64_t)blockIdx.x * nblocks;
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < nblocks; c0 += 256 * kItems) {
        const int64_t j = c0 + (int64_t)tid * kItems;
        int32_t v[kItems];
        int32_t s = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            v[k] = j + k < nblocks ? row[j + k] : 0;
            s += v[k];
        }
        int32_t incl = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        int32_t off = carry + incl - s, total = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            off += w < wid ? wsum[w] : 0;
            total += wsum[w];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (j + k < nblocks) row[j + k] = off;
            off += v[k];
        }
        carry += total;
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

struct Summary {
    int64_t n_groups;
    int32_t flag;
    int32_t pad;
    int64_t tot[kLevels];    // cells per level
};

__global__ void k_summary(int64_t n, const int32_t* __restrict__ gscan, const int32_t* __restrict__ flag,
                          const int32_t* __restrict__ tot, Summary* __restrict__ out) {
    if (threadIdx.x != 0) return;
    out->n_groups = gscan[n];
    out->flag = *flag;
    out->pad = 0;
    for (int L = 0; L < kLevels; ++L) out->tot[L] = tot[L];
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

struct LevelBase {
    int32_t off[kLevels + 1];   // first slot of each level; off[kLevels] = number of cells
};

// The cells starting at each particle (same tiling as k_levels): their
// level slot (level base + the block's offset + the rank among the block's
// cells of that level, by first particle) and, in preorder, their geometry,
// first index and key prefix; per slot the first particle, the preorder
// number and the slot of the first child (-1 for a leaf).
constexpr int kWords = kLvTile / 32;

__global__ __launch_bounds__(kLvThreads) void k_cells(int64_t n, int64_t nblocks, const uint64_t* __restrict__ keys,
                                                      const int8_t* __restrict__ delta,
                                                      const int8_t* __restrict__ leaflv,
                                                      const int32_t* __restrict__ start, LevelBase base,
                                                      const int32_t* __restrict__ blk, NodeGeo* __restrict__ geo,
                                                      int32_t* __restrict__ pfirst, uint64_t* __restrict__ prefix,
                                                      int32_t* __restrict__ sfirst, int32_t* __restrict__ spre,
                                                      int32_t* __restrict__ schild) {
    __shared__ uint32_t msk[kLevels][kWords];
    __shared__ int32_t wpre[kLevels][kWords];
    const int tid = threadIdx.x;
    const int64_t b0 = blockIdx.x * (int64_t)kLvTile;
    for (int q = tid; q < kLevels * kWords; q += kLvThreads) (&msk[0][0])[q] = 0u;
    __syncthreads();
    int d[kPer], ll[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int p = tid + q * kLvThreads;
        const int64_t s = b0 + p;
        d[q] = 0;
        ll[q] = 0;
        if (s < n) {
            d[q] = delta[s];
            ll[q] = leaflv[s];
            for (int L = d[q] + 1; L <= ll[q]; ++L) atomicOr(&msk[L][p >> 5], 1u << (p & 31));
        }
    }
    __syncthreads();
    if (tid < kLevels) {
        int32_t acc = 0;
        for (int w = 0; w < kWords; ++w) {
            wpre[tid][w] = acc;
            acc += __popc(msk[tid][w]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int p = tid + q * kLvThreads;
        const int64_t s = b0 + p;
        if (s >= n || ll[q] <= d[q]) continue;
        const int32_t st = start[s];
        const uint64_t k = keys[s];
        const uint32_t below = (1u << (p & 31)) - 1u;
        int32_t slot_next = -1;
        for (int L = ll[q]; L >= d[q] + 1; --L) {   // deepest first: each cell's first child is the one before
            const int32_t rank = wpre[L][p >> 5] + __popc(msk[L][p >> 5] & below);
            const int32_t slot = base.off[L] + blk[(int64_t)L * nblocks + blockIdx.x] + rank;
            const int32_t pre = st + (L - d[q] - 1);
            sfirst[slot] = (int32_t)s;
            spre[slot] = pre;
            schild[slot] = slot_next;
            slot_next = slot;
            const uint64_t pf = L == 0 ? 0ull : k >> (3 * (kMaxLevel - L));
            NodeGeo g;
            g.ix = compact3(pf >> 2);
            g.iy = compact3(pf >> 1);
            g.iz = compact3(pf);
            g.level_leaf = (uint32_t)L | (L == ll[q] ? 0x100u : 0u);
            geo[pre] = g;
            pfirst[pre] = (int32_t)s;
            prefix[pre] = pf;
        }
    }
}

// One level, deepest first, 4 lanes per cell.  A leaf's particles run to
// the first particle of the next cell in preorder; an inner cell's children
// are the next level's slots from its first child on, while their first
// particle lies before the first particle of the next slot of this level.
// Sums and counts are kept per slot; count, skip link and monopole go to
// the cell's preorder record, and the children get their parent.
constexpr int kMomLanes = 4;

__global__ __launch_bounds__(256) void k_moments(int32_t lo, int32_t hi, int32_t next_hi, int64_t n, int64_t nn,
                                                 const int32_t* __restrict__ sfirst, const int32_t* __restrict__ spre,
                                                 const int32_t* __restrict__ schild,
                                                 const int32_t* __restrict__ pfirst,
                                                 const int32_t* __restrict__ start, const double* __restrict__ px,
                                                 const double* __restrict__ py, const double* __restrict__ pz,
                                                 const double* __restrict__ pm, int32_t* __restrict__ scount,
                                                 double* __restrict__ sM, double* __restrict__ sX,
                                                 double* __restrict__ sY, double* __restrict__ sZ,
                                                 NodeRange* __restrict__ rng, double* __restrict__ oM,
                                                 double* __restrict__ oX, double* __restrict__ oY,
                                                 double* __restrict__ oZ, int32_t* __restrict__ leaf_of) {
    const int64_t i = lo + blockIdx.x * (int64_t)(256 / kMomLanes) + threadIdx.x / kMomLanes;
    const int j = threadIdx.x & (kMomLanes - 1);
    const bool on = i < hi;
    const int64_t c = on ? i : lo;
    const int32_t f = sfirst[c], pre = spre[c], ch = schild[c];
    double sm = 0, sx = 0, sy = 0, sz = 0;
    int64_t cnt = 0;
    if (on) {
        if (ch < 0) {
            const int64_t e = pre + 1 < nn ? pfirst[pre + 1] : n;
            for (int64_t s = f + j; s < e; s += kMomLanes) {
                const double mm = pm[s];
                sm += mm;
                sx += mm * px[s];
                sy += mm * py[s];
                sz += mm * pz[s];
                leaf_of[s] = pre;
            }
            cnt = j == 0 ? e - f : 0;
        } else {
            const int64_t lim = c + 1 < hi ? sfirst[c + 1] : n;   // first particle of the next cell of this level
            for (int64_t q = ch + j; q < next_hi && sfirst[q] < lim; q += kMomLanes) {
                sm += sM[q];
                sx += sX[q];
                sy += sY[q];
                sz += sZ[q];
                cnt += scount[q];
                rng[spre[q]].parent = pre;
            }
        }
    }
#pragma unroll
    for (int o = kMomLanes / 2; o >= 1; o >>= 1) {
        sm += __shfl_xor(sm, o, kMomLanes);
        sx += __shfl_xor(sx, o, kMomLanes);
        sy += __shfl_xor(sy, o, kMomLanes);
        sz += __shfl_xor(sz, o, kMomLanes);
        cnt += __shfl_xor(cnt, o, kMomLanes);
    }
    if (on && j == 0) {
        scount[c] = (int32_t)cnt;
        sM[c] = sm;
        sX[c] = sx;
        sY[c] = sy;
        sZ[c] = sz;
        const int64_t e = f + cnt;
        rng[pre].first = f;
        rng[pre].count = (int32_t)cnt;
        rng[pre].skip = e < n ? start[e] : (int32_t)nn;
        if (pre == 0) rng[pre].parent = -1;
        oM[pre] = sm;
        oX[pre] = sx / sm;
        oY[pre] = sy / sm;
        oZ[pre] = sz / sm;
    }
}

// A refitted tree (the structure held, the particles moved), one level,
// deepest first, 4 lanes per cell.  A leaf takes its particles at their
// periodic images nearest its dyadic centre; an inner cell takes its
// children's sums and boxes, each child moved as a whole by the whole
// number of box lengths that brings its box centre nearest the cell's
// centre.  The box is the min and max of those images per axis; the sums
// give the monopole.  Slot sums and boxes (sbox: lo xyz, hi xyz per slot)
// feed the next level up; monopoles and boxes go to the preorder records.
__global__ __launch_bounds__(256) void k_refit_level(int32_t lo, int32_t hi, int32_t next_hi, int64_t n,
                                                     const int32_t* __restrict__ sfirst,
                                                     const int32_t* __restrict__ spre,
                                                     const int32_t* __restrict__ schild,
                                                     const NodeGeo* __restrict__ geo,
                                                     const NodeRange* __restrict__ rng, const double* __restrict__ px,
                                                     const double* __restrict__ py, const double* __restrict__ pz,
                                                     const double* __restrict__ pm, double* __restrict__ sM,
                                                     double* __restrict__ sX, double* __restrict__ sY,
                                                     double* __restrict__ sZ, double* __restrict__ sbox,
                                                     double* __restrict__ oM, double* __restrict__ oX,
                                                     double* __restrict__ oY, double* __restrict__ oZ,
                                                     double* __restrict__ clo, double* __restrict__ chi) {
    const int64_t i = lo + blockIdx.x * (int64_t)(256 / kMomLanes) + threadIdx.x / kMomLanes;
    const int j = threadIdx.x & (kMomLanes - 1);
    const bool on = i < hi;
    const int64_t c = on ? i : lo;
    const int32_t f = sfirst[c], pre = spre[c], ch = schild[c];
    const NodeGeo g = geo[pre];
    const int lv = (int)(g.level_leaf & 0xffu);
    const double cref[3] = {ldexp((double)g.ix + 0.5, -lv), ldexp((double)g.iy + 0.5, -lv),
                            ldexp((double)g.iz + 0.5, -lv)};
    double sm = 0, sv[3] = {0, 0, 0}, bl[3], bh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bl[a] = INFINITY;
        bh[a] = -INFINITY;
    }
    if (on) {
        if (ch < 0) {
            const int64_t e = f + (int64_t)rng[pre].count;
            for (int64_t s = f + j; s < e; s += kMomLanes) {
                const double mm = pm[s];
                const double u[3] = {px[s], py[s], pz[s]};
                sm += mm;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double v = u[a] - rint(u[a] - cref[a]);
                    sv[a] += mm * v;
                    bl[a] = v < bl[a] ? v : bl[a];
                    bh[a] = v > bh[a] ? v : bh[a];
                }
            }
        } else {
            const int64_t lim = c + 1 < hi ? sfirst[c + 1] : n;
            for (int64_t q = ch + j; q < next_hi && sfirst[q] < lim; q += kMomLanes) {
                const double mq = sM[q];
                const double sq[3] = {sX[q], sY[q], sZ[q]};
                sm += mq;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double l = sbox[q * 6 + a], h = sbox[q * 6 + 3 + a];
                    const double sh = rint((l + h) * 0.5 - cref[a]);
                    const double vl = l - sh, vh = h - sh;
                    bl[a] = vl < bl[a] ? vl : bl[a];
                    bh[a] = vh > bh[a] ? vh : bh[a];
                    sv[a] += sq[a] - sh * mq;
                }
            }
        }
    }
#pragma unroll
    for (int o = kMomLanes / 2; o >= 1; o >>= 1) {
        sm += __shfl_xor(sm, o, kMomLanes);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sv[a] += __shfl_xor(sv[a], o, kMomLanes);
            const double l = __shfl_xor(bl[a], o, kMomLanes), h = __shfl_xor(bh[a], o, kMomLanes);
            bl[a] = l < bl[a] ? l : bl[a];
            bh[a] = h > bh[a] ? h : bh[a];
        }
    }
    if (on && j == 0) {
        sM[c] = sm;
        sX[c] = sv[0];
        sY[c] = sv[1];
        sZ[c] = sv[2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            sbox[c * 6 + a] = bl[a];
            sbox[c * 6 + 3 + a] = bh[a];
            clo[(int64_t)pre * 3 + a] = bl[a];
            chi[(int64_t)pre * 3 + a] = bh[a];
        }
        oM[pre] = sm;
        oX[pre] = sv[0] / sm;
        oY[pre] = sv[1] / sm;
        oZ[pre] = sv[2] / sm;
    }
}

// A cell's 16-byte packed record.
__device__ __forceinline__ uint4 pack16(const NodeGeo& g, const NodeRange& r) {
    const uint32_t sk = (uint32_t)r.skip;
    const uint32_t lv = g.level_leaf & 0xffu;
    const bool leaf = (g.level_leaf >> 8) & 1u;
    uint4 pk;
    pk.x = g.ix | ((sk & 0x7ffu) << 21);
    pk.y = g.iy | (((sk >> 11) & 0x7ffu) << 21);
    pk.z = g.iz | (((sk >> 22) & 0x3ffu) << 21);
    pk.w = lv | (leaf ? 0x20u : 0u) | ((uint32_t)(r.count < (int32_t)kPackCountMax ? r.count : (int32_t)kPackCountMax) << 6);
    return pk;
}

// The 8-byte walk record of each cell (preorder).
__global__ void k_pack(int64_t nn, const NodeGeo* __restrict__ geo, const NodeRange* __restrict__ rng,
                       uint2* __restrict__ pack) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nn) return;
    const NodeGeo g = geo[c];
    const NodeRange r = rng[c];
    const uint32_t lv = g.level_leaf & 0xffu;
    const uint32_t leaf = (g.level_leaf >> 8) & 1u;
    const uint32_t oct = ((g.ix & 1u) << 2) | ((g.iy & 1u) << 1) | (g.iz & 1u);
    const uint32_t cnt = r.count < (int32_t)kWalkCountMax ? (uint32_t)r.count : kWalkCountMax;
    pack[c] = make_uint2(lv | (leaf << 5) | (oct << 6) | (cnt << 9), (uint32_t)r.skip);
}

// The walk record of each cell of a refitted tree (preorder): the packed
// record, and the box rounded outward to multiples of q = 2^-(level + 10),
// K = floor(lo / q) and ceil(hi / q) (exact), stored as offsets from the
// centre's multiple ic * 1024 + 512 when both fit 16 bits.
__global__ void k_refit_pack(int64_t nn, const NodeGeo* __restrict__ geo, const NodeRange* __restrict__ rng,
                             const double* __restrict__ clo, const double* __restrict__ chi,
                             RefitCell* __restrict__ out) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nn) return;
    const NodeGeo g = geo[c];
    const int e = (int)(g.level_leaf & 0xffu) + kRefitShift;
    const uint32_t ic[3] = {g.ix, g.iy, g.iz};
    RefitCell r;
    r.pk = pack16(g, rng[c]);
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t kc = (int64_t)ic[a] * (1 << kRefitShift) + (1 << (kRefitShift - 1));
        const int64_t kl = (int64_t)floor(ldexp(clo[c * 3 + a], e)) - kc;
        const int64_t kh = (int64_t)ceil(ldexp(chi[c * 3 + a], e)) - kc;
        ok = ok && kl >= -kRefitMaxOff && kh <= kRefitMaxOff;
        r.b[a] = (int32_t)(((uint32_t)(uint16_t)(int16_t)kl) | ((uint32_t)(uint16_t)(int16_t)kh << 16));
    }
    r.b[3] = ok ? 1 : 0;
    out[c] = r;
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
// j, j + 16, ... (min and max are exact in any order).  In a refitted tree
// (REFIT) each position is first moved to its periodic image nearest the
// group's first particle.
constexpr int kBoxLanes = 16;

template <bool REFIT>
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
        const double r[3] = {px[f], py[f], pz[f]};
        for (int32_t q = j; q < cnt; q += kBoxLanes) {
            double v[3] = {px[f + q], py[f + q], pz[f + q]};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (REFIT) v[k] = v[k] - rint(v[k] - r[k]);
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

}  // namespace

bool build_cells_and_groups(Tree& t, int32_t* d_flag, hipStream_t st) {
    const int64_t n = t.n;
    const int B = 256;
    const int64_t nblocks = (n + kLvTile - 1) / kLvTile;
    // per-particle levels, chain lengths and group starts; per-block cell counts
    DevBuf<int8_t> delta(n, st), leaflv(n, st);
    DevBuf<int32_t> start(n + 1, st), mark(n + 1, st), blk((kLevels + 2) * nblocks, st), tot(kLevels + 2, st);
    DevBuf<Summary> dsum(1, st);
    hipLaunchKernelGGL(k_levels, dim3((unsigned)nblocks), dim3(kLvThreads), 0, st, n, t.keys.get(), t.n_leaf,
                       t.n_group, nblocks, delta.get(), leaflv.get(), start.get(), mark.get(), blk.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_level_scan, dim3(kLevels + 2), dim3(256), 0, st, nblocks, blk.get(), tot.get());
    SRF_HIP(hipGetLastError());
    // preorder number of each chain's first cell, group number of each group start
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nblocks), dim3(kLvThreads), 0, st, n, nblocks, start.get(),
                       mark.get(), blk.get(), tot.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_summary, dim3(1), dim3(64), 0, st, n, mark.get(), d_flag, tot.get(), dsum.get());
    SRF_HIP(hipGetLastError());
    // the one synchronisation: sizes and the device's check of the inputs
    Summary hs;
    SRF_HIP(hipMemcpyAsync(&hs, dsum.get(), sizeof(Summary), hipMemcpyDeviceToHost, st));
    SRF_HIP(hipStreamSynchronize(st));
    // the cells below read the sorted positions, gathered on the second stream
    if (t.gathered) SRF_HIP(hipStreamWaitEvent(st, t.gathered, 0));
    if (hs.flag & 1) fail(SRF_EDOMAIN, "non-finite particle position");
    if (hs.flag & 2) fail(SRF_EDOMAIN, "particle mass not finite and > 0");
    if (hs.flag & 8) return false;   // the order is incomplete (see build_sorted)
    // (a level holds fewer than 2^31 cells: its per-block counts are exact
    // int32 sums of counts below n; the total is checked here)
    LevelBase base;
    int64_t acc = 0;
    int max_level = 0;
    for (int L = 0; L < kLevels; ++L) {
        base.off[L] = (int32_t)(acc < INT32_MAX ? acc : INT32_MAX);
        acc += hs.tot[L];
        if (hs.tot[L] > 0) max_level = L;
    }
    if (acc > (int64_t)INT32_MAX - 1)
        fail(SRF_EINVAL, "the tree would hold " + std::to_string(acc) + " cells, past 32-bit cell indices");
    base.off[kLevels] = (int32_t)acc;
    const int64_t nn = acc, ng = hs.n_groups;
    t.n_nodes = nn;
    t.n_groups = ng;
    t.max_level = max_level;

    // cells: slots and geometry, then counts, moments and links bottom-up
    t.geo.alloc(nn, st);
    t.range.alloc(nn, st);
    t.pack.alloc(nn, st);
    t.prefix.alloc(nn, st);
    t.nM.alloc(nn, st);
    t.nX.alloc(nn, st);
    t.nY.alloc(nn, st);
    t.nZ.alloc(nn, st);
    t.leaf_of.alloc(n, st);
    t.sfirst.alloc(nn, st);
    t.spre.alloc(nn, st);
    t.schild.alloc(nn, st);
    for (int L = 0; L <= kLevels; ++L) t.level_off[L] = base.off[L];
    int32_t* sfirst = t.sfirst.get();
    int32_t* spre = t.spre.get();
    int32_t* schild = t.schild.get();
    DevBuf<int32_t> pfirst(nn, st), scount(nn, st);
    DevBuf<double> sM(nn, st), sX(nn, st), sY(nn, st), sZ(nn, st);
    // the point after which the second stream may build the groups
    hipStream_t aux = aux_stream();
    SRF_HIP(hipEventCreateWithFlags(&t.sized, hipEventDisableTiming));
    SRF_HIP(hipEventCreateWithFlags(&t.grouped, hipEventDisableTiming));
    SRF_HIP(hipEventRecord(t.sized, st));

    hipLaunchKernelGGL(k_cells, dim3((unsigned)nblocks), dim3(kLvThreads), 0, st, n, nblocks, t.keys.get(),
                       delta.get(), leaflv.get(), start.get(), base, blk.get(), t.geo.get(), pfirst.get(),
                       t.prefix.get(), sfirst, spre, schild);
    SRF_HIP(hipGetLastError());
    for (int L = max_level; L >= 0; --L) {
        const int32_t lo = base.off[L], hi = base.off[L + 1];
        if (hi <= lo) continue;
        const int32_t next_hi = L < kMaxLevel ? base.off[L + 2] : hi;
        hipLaunchKernelGGL(k_moments, dim3(grid_for(hi - lo, 256 / kMomLanes, 1 << 30)), dim3(256), 0, st, lo, hi,
                           next_hi, n, nn, sfirst, spre, schild, pfirst.get(), start.get(),
                           t.px.get(), t.py.get(), t.pz.get(), t.pm.get(), scount.get(), sM.get(), sX.get(), sY.get(),
                           sZ.get(), t.range.get(), t.nM.get(), t.nX.get(), t.nY.get(), t.nZ.get(), t.leaf_of.get());
        SRF_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nn, B, 1 << 30)), dim3(B), 0, st, nn, t.geo.get(), t.range.get(),
                       t.pack.get());
    SRF_HIP(hipGetLastError());

    // groups (from the marks and the sorted positions alone) on the second
    // stream, beside the cells (queued after them: the cells are the longer
    // chain)
    t.gfirst.alloc(ng, st);
    t.gcount.alloc(ng, st);
    t.glo.alloc(ng * 3, st);
    t.ghi.alloc(ng * 3, st);
    // on every way out (an error included) `grouped` marks all the work
    // queued on the second stream, and the build's stream waits for it
    // before the marks are freed (declared after them, so destroyed first)
    struct JoinAtExit {
        hipStream_t st, aux;
        hipEvent_t e;
        ~JoinAtExit() {
            (void)hipEventRecord(e, aux);
            (void)hipStreamWaitEvent(st, e, 0);
        }
    } join{st, aux, t.grouped};
    SRF_HIP(hipStreamWaitEvent(aux, t.sized, 0));
    hipLaunchKernelGGL(k_group_write, dim3(grid_for(n, B, 1 << 30)), dim3(B), 0, aux, n, mark.get(), t.gfirst.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_group_count, dim3(grid_for(ng, B, 1 << 30)), dim3(B), 0, aux, ng, n, t.gfirst.get(),
                       t.gcount.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_group_bbox<false>, dim3(grid_for(ng, 256 / kBoxLanes, 1 << 30)), dim3(256), 0, aux, ng,
                       t.gfirst.get(), t.gcount.get(), t.px.get(), t.py.get(), t.pz.get(), t.glo.get(), t.ghi.get());
    SRF_HIP(hipGetLastError());
    return true;
}

void refit_cells_and_groups(Tree& t, hipStream_t st) {
    const int64_t n = t.n, nn = t.n_nodes, ng = t.n_groups;
    if (!t.clo.get()) {
        t.clo.alloc(nn * 3, st);
        t.chi.alloc(nn * 3, st);
    }
    DevBuf<double> sM(nn, st), sX(nn, st), sY(nn, st), sZ(nn, st), sbox(nn * 6, st);
    for (int L = t.max_level; L >= 0; --L) {
        const int32_t lo = t.level_off[L], hi = t.level_off[L + 1];
        if (hi <= lo) continue;
        const int32_t next_hi = L < kMaxLevel ? t.level_off[L + 2] : hi;
        hipLaunchKernelGGL(k_refit_level, dim3(grid_for(hi - lo, 256 / kMomLanes, 1 << 30)), dim3(256), 0, st, lo,
                           hi, next_hi, n, t.sfirst.get(), t.spre.get(), t.schild.get(), t.geo.get(), t.range.get(),
                           t.px.get(), t.py.get(), t.pz.get(), t.pm.get(), sM.get(), sX.get(), sY.get(), sZ.get(),
                           sbox.get(), t.nM.get(), t.nX.get(), t.nY.get(), t.nZ.get(), t.clo.get(), t.chi.get());
        SRF_HIP(hipGetLastError());
    }
    if (!t.rpack.get()) t.rpack.alloc(nn, st);
    hipLaunchKernelGGL(k_refit_pack, dim3(grid_for(nn, 256, 1 << 30)), dim3(256), 0, st, nn, t.geo.get(),
                       t.range.get(), t.clo.get(), t.chi.get(), t.rpack.get());
    SRF_HIP(hipGetLastError());
    if (ng > 0) {
        hipLaunchKernelGGL(k_group_bbox<true>, dim3(grid_for(ng, 256 / kBoxLanes, 1 << 30)), dim3(256), 0, st, ng,
                           t.gfirst.get(), t.gcount.get(), t.px.get(), t.py.get(), t.pz.get(), t.glo.get(),
                           t.ghi.get());
        SRF_HIP(hipGetLastError());
    }
}

}  // namespace srf
