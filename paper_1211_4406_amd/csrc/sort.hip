// Steps a1-a2: periodic wrap, 63-bit Morton keys, stable LSD radix sort of
// (key, input index), gather of the sorted SoA particle arrays.
//
// The sort orders (key, input index) with passes over 32-bit words.  Four
// stable passes order (high word; index) by the high word.  Particles that
// share their high word with a neighbour then form runs, and each run is
// ordered by (low word, index): every member counts the members that come
// before it (runs hold at most kRunMax particles; a longer run, which needs
// more than kRunMax particles in one cube of side 2^-10 of the box, makes
// the caller sort again in full).  The full sort: four passes order (low word; high
// word, index) by the low word, four more (high word; index) by the high
// word.  Both give the order of (key, input index), that of eight passes
// over the whole 64-bit key.  The sorted keys are recomputed from the
// sorted positions by the final gather.
#include "common.h"

namespace srf {
namespace {

// Wrap into [0,1): u = v - floor(v); a tiny negative v rounds to u == 1,
// which is the same point as 0.
__device__ __forceinline__ double wrap01(double v) {
    double u = v - floor(v);
    return u == 1.0 ? 0.0 : u;
}

// Spread the low 21 bits of v so that bit b lands on bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ uint64_t grid21(double u) {
    double c = floor(u * 2097152.0);  // 2^21, exact product
    c = c > 2097151.0 ? 2097151.0 : c;
    c = c >= 0.0 ? c : 0.0;           // also maps NaN to 0 (flagged separately)
    return (uint64_t)c;
}

__global__ void k_keys(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                       const double* __restrict__ z, int64_t ps, const double* __restrict__ m, int64_t ms,
                       uint32_t* __restrict__ klo, uint32_t* __restrict__ khi, int32_t* __restrict__ vals,
                       int32_t* __restrict__ flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = x[i * ps], b = y[i * ps], c = z[i * ps], mm = m[i * ms];
    int bad = 0;
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) bad |= 1;
    if (!(isfinite(mm) && mm > 0.0)) bad |= 2;
    if (bad) atomicOr(flag, bad);
    uint64_t kx = grid21(wrap01(a)), ky = grid21(wrap01(b)), kz = grid21(wrap01(c));
    const uint64_t key = (spread3(kx) << 2) | (spread3(ky) << 1) | spread3(kz);
    klo[i] = (uint32_t)key;
    khi[i] = (uint32_t)(key >> 32);
    vals[i] = (int32_t)i;
}

// ------------------------------------------------------------- radix sort
// Eight LSD passes of 8 bits over the 64-bit key.  A block sorts a tile of
// kTile keys; its wave w owns the kWaveKeys consecutive keys starting at
// w * kWaveKeys, read in rounds of 64 (item r of lane l is key
// w * kWaveKeys + 64 r + l), so a key's rank within its wave needs no
// block-wide barrier.  Each pass: per-tile digit counts (k_hist), their
// exclusive scan over the tiles of each digit (k_digit_scan), and the stable
// scatter (k_scatter), which adds the scan over digits itself.
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 16;   // keys per thread: tiles of 4096 (8 and 12 measured no faster at 2^24)
constexpr int kWaveKeys = 64 * kItems;
constexpr int kTile = kThreads * kItems;  // keys per block
constexpr int kDigits = 256;
static_assert(kThreads == kDigits, "one digit per thread in the per-digit steps");

__global__ __launch_bounds__(kThreads) void k_hist(int64_t n, const uint32_t* __restrict__ keys, int shift,
                                                   int64_t tiles, int32_t* __restrict__ counts) {
    __shared__ int32_t h[kWaves][kDigits];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) h[w][tid] = 0;
    __syncthreads();
    const int64_t base = blockIdx.x * (int64_t)kTile + wid * kWaveKeys + lane;
    uint32_t k[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + 64 * r;
        k[r] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r)
        if (base + 64 * r < n) atomicAdd(&h[wid][(k[r] >> shift) & 0xff], 1);
    __syncthreads();
    int32_t c = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) c += h[w][tid];
    counts[(int64_t)tid * tiles + blockIdx.x] = c;
}

// Exclusive scan of one digit's row of per-tile counts (block = digit), in
// place; the digit's total goes to dtot.
__global__ __launch_bounds__(kThreads) void k_digit_scan(int64_t tiles, int32_t* __restrict__ counts,
                                                         int32_t* __restrict__ dtot) {
    constexpr int kPer = 4;
    __shared__ int32_t wsum[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int32_t* row = counts + (int64_t)blockIdx.x * tiles;
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < tiles; c0 += kThreads * kPer) {
        const int64_t j = c0 + (int64_t)tid * kPer;
        int32_t v[kPer];
        int32_t s = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            v[k] = j + k < tiles ? row[j + k] : 0;
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
        for (int w = 0; w < kWaves; ++w) {
            off += w < wid ? wsum[w] : 0;
            total += wsum[w];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (j + k < tiles) row[j + k] = off;
            off += v[k];
        }
        carry += total;
    }
    if (tid == 0) dtot[blockIdx.x] = carry;
}

// Stable scatter of one tile.  Ranking: in each round the lanes holding the
// same digit are found by eight ballots; a key's rank is its wave's running
// count of that digit (an LDS counter, advanced by the lowest such lane)
// plus the number of such lanes below it.  Tile position: digits in order,
// within a digit the waves in order, then the rank.  The tile is reordered
// in LDS so that each digit's run is written contiguously.
template <bool V2>
__global__ __launch_bounds__(kThreads) void k_scatter(int64_t n, const uint32_t* __restrict__ kin,
                                                      const int32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                      int32_t* __restrict__ vout, const uint32_t* __restrict__ v2in,
                                                      uint32_t* __restrict__ v2out, int shift, int64_t tiles,
                                                      const int32_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ dtot) {
    __shared__ int32_t wc[kWaves][kDigits];   // running counts, then the waves' exclusive prefix
    __shared__ int32_t toff[kDigits];         // tile-local exclusive offset of each digit
    __shared__ int32_t gdst[kDigits];         // global position of the tile's first key of each digit
    __shared__ int32_t wsum[kWaves][2];
    __shared__ uint32_t skey[kTile];
    __shared__ int32_t sval[kTile];
    __shared__ uint32_t sval2[V2 ? kTile : 1];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wc[w][tid] = 0;
    const int32_t tile_base = offsets[(int64_t)tid * tiles + blockIdx.x];
    const int32_t digit_total = dtot[tid];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t wbase = blockIdx.x * (int64_t)kTile + wid * kWaveKeys + lane;
    uint32_t key[kItems], val2[kItems];
    int32_t val[kItems], rank[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = wbase + 64 * r;
        key[r] = i < n ? kin[i] : 0u;
        val[r] = i < n ? vin[i] : 0;
        val2[r] = (V2 && i < n) ? v2in[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const bool valid = wbase + 64 * r < n;
        const int d = (int)((key[r] >> shift) & 0xff);
        // lanes holding the same digit (invalid lanes match only each other)
        uint64_t peers = __ballot(valid);
        if (!valid) peers = ~peers;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const int lower = __popcll(peers & lt);
        int32_t old = 0;
        if (valid) old = wc[wid][d];
        rank[r] = old + lower;
        if (valid && lower == 0) wc[wid][d] = old + __popcll(peers);
        // the next round's reads must see this round's counter (one wave:
        // LDS operations complete in order; this keeps the compiler's too)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    // per digit (one per thread): the waves' exclusive prefix and the tile
    // total, then exclusive scans over digits of the tile totals and of the
    // global digit totals
    int32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int32_t c = wc[w][tid];
        wc[w][tid] = tot;
        tot += c;
    }
    int32_t it = tot, ig = digit_total;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t ut = __shfl_up(it, o, 64), ug = __shfl_up(ig, o, 64);
        if (lane >= o) {
            it += ut;
            ig += ug;
        }
    }
    if (lane == 63) {
        wsum[wid][0] = it;
        wsum[wid][1] = ig;
    }
    __syncthreads();
    int32_t ot = it - tot, og = ig - digit_total;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        if (w < wid) {
            ot += wsum[w][0];
            og += wsum[w][1];
        }
    }
    toff[tid] = ot;
    gdst[tid] = og + tile_base;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (wbase + 64 * r >= n) continue;
        const int d = (int)((key[r] >> shift) & 0xff);
        const int p = toff[d] + wc[wid][d] + rank[r];
        if ((unsigned)p < (unsigned)kTile) {
            skey[p] = key[r];
            sval[p] = val[r];
            if (V2) sval2[p] = val2[r];
        }
    }
    __syncthreads();
    const int64_t tbase = blockIdx.x * (int64_t)kTile;
    const int cnt = (int)((n - tbase) < kTile ? (n - tbase) : kTile);
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int p = r * kThreads + tid;
        if (p < cnt) {
            const uint32_t k = skey[p];
            const int d = (int)((k >> shift) & 0xff);
            const int64_t dst = (int64_t)gdst[d] + (p - toff[d]);
            if ((uint64_t)dst < (uint64_t)n) {   // always, by construction; never a stray store
                kout[dst] = k;
                vout[dst] = sval[p];
                if (V2) v2out[dst] = sval2[p];
            }
        }
    }
}

// ------------------------------------------------------------- runs
// After the high-word passes: positions whose high word a neighbour
// shares (mark 1), compacted in order with their low words, and each such
// run put in (low word, index) order by counting.
constexpr int64_t kRunMax = 1024;
constexpr int kRunGrid = 4096;   // blocks of the kernels that loop over the run members

__device__ __forceinline__ bool in_run(const uint32_t* __restrict__ hi, int64_t n, int64_t s) {
    const uint32_t h = hi[s];
    return (s > 0 && hi[s - 1] == h) || (s + 1 < n && hi[s + 1] == h);
}

// The marks, and one past the last marked position: the largest over the
// blocks, kept in kRunSlots slots (block b in slot b mod kRunSlots, zeroed
// first) so that few atomics meet on one address.
constexpr int kRunSlots = 1024;
__global__ __launch_bounds__(256) void k_run_mark(int64_t n, const uint32_t* __restrict__ hi,
                                                  int32_t* __restrict__ mark, int32_t* __restrict__ blast) {
    __shared__ int32_t last;
    if (threadIdx.x == 0) last = 0;
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool m = s < n && in_run(hi, n, s);
    if (s < n) mark[s] = m ? 1 : 0;
    // the wave's last marked lane, then the block's
    const uint64_t b = __ballot(m);
    if (b && (threadIdx.x & 63) == 0)
        atomicMax(&last, (int32_t)(s + (63 - __clzll((long long)b)) + 1));
    __syncthreads();
    if (threadIdx.x == 0 && last > 0) atomicMax(&blast[blockIdx.x & (kRunSlots - 1)], last);
}

// rc[0] = one past the last marked position (the largest slot), so that
// the scan of the marks can stop there and costs nothing when no two
// particles share a high word; rc[1] = 0 (the number of marks, written by
// the compaction).  One block, one slot per thread.
__global__ __launch_bounds__(kRunSlots) void k_run_end(const int32_t* __restrict__ blast, int32_t* __restrict__ rc) {
    __shared__ int32_t wmax[kRunSlots / 64];
    int32_t v = blast[threadIdx.x];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int32_t u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t r = 0;
        for (int w = 0; w < kRunSlots / 64; ++w) r = wmax[w] > r ? wmax[w] : r;
        rc[0] = r;
        rc[1] = 0;
    }
}

// `at`: exclusive scan of the marks before rc[0]; the last marked position
// writes their number to rc[1] (zeroed first).
__global__ void k_run_compact(const int32_t* __restrict__ rc_end, const uint32_t* __restrict__ hi,
                              const int32_t* __restrict__ idx, const uint32_t* __restrict__ klo,
                              const int32_t* __restrict__ at, uint32_t* __restrict__ clo,
                              uint32_t* __restrict__ chi, int32_t* __restrict__ cidx, int32_t* __restrict__ cpos,
                              int32_t* __restrict__ rc_count, int64_t n) {
    const int64_t end = *rc_end;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < end; s += (int64_t)gridDim.x * blockDim.x) {
        if (!in_run(hi, n, s)) continue;
        const int64_t j = at[s];
        const int32_t i = idx[s];
        clo[j] = klo[i];
        chi[j] = hi[s];
        cidx[j] = i;
        cpos[j] = (int32_t)s;
        if (s == end - 1) *rc_count = (int32_t)(j + 1);
    }
}

// Run starts in the compacted array: rid[j] = 1 where run j begins (then
// scanned into run numbers).
__global__ void k_run_starts(const int32_t* __restrict__ md, const uint32_t* __restrict__ chi,
                             int32_t* __restrict__ rid) {
    const int64_t m = *md;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        rid[j] = (j == 0 || chi[j] != chi[j - 1]) ? 1 : 0;
}

// rstart[r] = first member of run r (rid: exclusive scan of the starts,
// so rid[j] is the run number of a start j and rid[m] the number of runs);
// rstart[number of runs] = m.
__global__ void k_run_index(const int32_t* __restrict__ md, const uint32_t* __restrict__ chi,
                            const int32_t* __restrict__ rid, int32_t* __restrict__ rstart) {
    const int64_t m = *md;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= m; j += (int64_t)gridDim.x * blockDim.x) {
        if (j == m) {
            rstart[rid[m]] = (int32_t)m;
        } else if (j == 0 || chi[j] != chi[j - 1]) {
            rstart[rid[j]] = (int32_t)j;
        }
    }
}

// Member j of a run [r0, r1) of the compacted array goes to r0 + the number
// of members with a smaller (low word, index); the members' positions in
// the sorted array are the run's positions, in order.  A run longer than
// kRunMax sets bit 3 of *flag instead.
__global__ void k_run_rank(int64_t n, const int32_t* __restrict__ md, const uint32_t* __restrict__ clo,
                           const int32_t* __restrict__ cidx, const int32_t* __restrict__ cpos,
                           const int32_t* __restrict__ rid, const int32_t* __restrict__ rstart,
                           int32_t* __restrict__ perm, int32_t* __restrict__ flag) {
    const int64_t m = *md;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = rid[j + 1] - 1;   // starts in [0, j], less one: j's run
        const int32_t r0 = rstart[r], r1 = rstart[r + 1];
        if (r1 - r0 > kRunMax) {
            atomicOr(flag, 8);
            continue;
        }
        const uint32_t lo = clo[j];
        const int32_t id = cidx[j];
        int32_t rank = 0;
#pragma unroll 4
        for (int32_t k = r0; k < r1; ++k) {
            const uint32_t l = clo[k];
            rank += (l < lo || (l == lo && cidx[k] < id)) ? 1 : 0;
        }
        const int32_t p = cpos[r0 + rank];
        if ((uint64_t)p < (uint64_t)n) perm[p] = id;
    }
}

// The sorted particles and, with KEYS, their keys computed again from the
// wrapped positions exactly as k_keys computed them.
template <bool KEYS>
__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ x,
                         const double* __restrict__ y, const double* __restrict__ z, int64_t ps,
                         const double* __restrict__ m, int64_t ms, double* __restrict__ px, double* __restrict__ py,
                         double* __restrict__ pz, double* __restrict__ pm, uint64_t* __restrict__ keys) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t i = perm[s];
    const double u = wrap01(x[i * ps]), v = wrap01(y[i * ps]), w = wrap01(z[i * ps]);
    px[s] = u;
    py[s] = v;
    pz[s] = w;
    pm[s] = m[i * ms];
    if (KEYS) keys[s] = (spread3(grid21(u)) << 2) | (spread3(grid21(v)) << 1) | spread3(grid21(w));
}

// The sorted keys from the sorted high words and the low words k_keys left
// in input order.
__global__ void k_sorted_keys(int64_t n, const int32_t* __restrict__ perm, const uint32_t* __restrict__ hi,
                              const uint32_t* __restrict__ lo, uint64_t* __restrict__ keys) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    keys[s] = ((uint64_t)hi[s] << 32) | lo[perm[s]];
}

// The same gather for a tree reused at new positions, with the input checks
// of k_keys; without masses (m == nullptr) only the positions are gathered.
__global__ void k_gather_checked(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ x,
                                 const double* __restrict__ y, const double* __restrict__ z, int64_t ps,
                                 const double* __restrict__ m, int64_t ms, double* __restrict__ px,
                                 double* __restrict__ py, double* __restrict__ pz, double* __restrict__ pm,
                                 int32_t* __restrict__ flag) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t i = perm[s];
    const double a = x[i * ps], b = y[i * ps], c = z[i * ps];
    int bad = (isfinite(a) && isfinite(b) && isfinite(c)) ? 0 : 1;
    px[s] = wrap01(a);
    py[s] = wrap01(b);
    pz[s] = wrap01(c);
    if (m) {
        const double mm = m[i * ms];
        if (!(isfinite(mm) && mm > 0.0)) bad |= 2;
        pm[s] = mm;
    }
    if (bad) atomicOr(flag, bad);
}

}  // namespace

void gather_refit(const Tree& t, const double* x, const double* y, const double* z, int64_t ps, const double* m,
                  int64_t ms, int32_t* d_flag, double* px, double* py, double* pz, double* pm, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_checked, dim3(grid_for(t.n, 256, 1 << 30)), dim3(256), 0, st, t.n, t.perm.get(), x,
                       y, z, ps, m, ms, px, py, pz, pm, d_flag);
    SRF_HIP(hipGetLastError());
}

void build_sorted(Tree& t, const double* x, const double* y, const double* z, int64_t ps, const double* m,
                  int64_t ms, int32_t* d_flag, bool full, hipStream_t st) {
    const int64_t n = t.n;
    const int B = 256;
    DevBuf<uint32_t> ka(n, st), kb(n, st), ha(n, st), hb(n, st);
    DevBuf<int32_t> vb(n, st);
    t.keys.alloc(n, st);
    t.perm.alloc(n, st);
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, B, 1 << 30)), dim3(B), 0, st, n, x, y, z, ps, m, ms, ka.get(),
                       ha.get(), t.perm.get(), d_flag);
    SRF_HIP(hipGetLastError());
    const int64_t tiles = (n + kTile - 1) / kTile;
    DevBuf<int32_t> counts(kDigits * tiles, st);
    DevBuf<int32_t> dtot(kDigits, st);
    // one stable pass of 8 bits over the words k (with index v and, for the
    // low word, the high word h carried along)
    auto pass = [&](int shift, const uint32_t* k, uint32_t* k2, const int32_t* v, int32_t* v2, const uint32_t* h,
                    uint32_t* h2) {
        hipLaunchKernelGGL(k_hist, dim3((unsigned)tiles), dim3(kThreads), 0, st, n, k, shift, tiles, counts.get());
        SRF_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_digit_scan, dim3(kDigits), dim3(kThreads), 0, st, tiles, counts.get(), dtot.get());
        SRF_HIP(hipGetLastError());
        if (h)
            hipLaunchKernelGGL(k_scatter<true>, dim3((unsigned)tiles), dim3(kThreads), 0, st, n, k, v, k2, v2, h, h2,
                               shift, tiles, counts.get(), dtot.get());
        else
            hipLaunchKernelGGL(k_scatter<false>, dim3((unsigned)tiles), dim3(kThreads), 0, st, n, k, v, k2, v2,
                               (const uint32_t*)nullptr, (uint32_t*)nullptr, shift, tiles, counts.get(), dtot.get());
        SRF_HIP(hipGetLastError());
    };
    // full: the low word first, passes a -> b -> a -> b -> a (pairs of
    // passes return to the first buffers), then the high word, already in
    // that order, in ha; otherwise the high word alone, then the runs
    if (full) {
        for (int p = 0; p < 4; p += 2) {
            pass(8 * p, ka.get(), kb.get(), t.perm.get(), vb.get(), ha.get(), hb.get());
            pass(8 * (p + 1), kb.get(), ka.get(), vb.get(), t.perm.get(), hb.get(), ha.get());
        }
    }
    for (int p = 0; p < 4; p += 2) {
        pass(8 * p, ha.get(), hb.get(), t.perm.get(), vb.get(), nullptr, nullptr);
        pass(8 * (p + 1), hb.get(), ha.get(), vb.get(), t.perm.get(), nullptr, nullptr);
    }
    if (!full) {
        const dim3 grid(grid_for(n, B, 1 << 30));
        DevBuf<int32_t> at(n + 1, st), rc(2, st), blast(kRunSlots, st);   // rc: end of the marks, their number
        fill_i32(blast.get(), 0, kRunSlots, st);
        hipLaunchKernelGGL(k_run_mark, grid, dim3(B), 0, st, n, ha.get(), at.get(), blast.get());
        SRF_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_run_end, dim3(1), dim3(kRunSlots), 0, st, blast.get(), rc.get());
        SRF_HIP(hipGetLastError());
        exclusive_scan_i32_counted(at.get(), n, rc.get(), st);
        // the compacted runs: low word in kb, high word in hb, index in vb, position in cpos
        DevBuf<int32_t> cpos(n, st);
        // the kernels below loop over a count held on the device: a grid of
        // kRunGrid blocks covers any count, and costs little when it is 0
        // (the ranking, whose members' work varies with their run's length,
        // keeps one thread per position)
        const dim3 rgrid(grid_for(n + 1, B, kRunGrid));
        hipLaunchKernelGGL(k_run_compact, rgrid, dim3(B), 0, st, rc.get(), ha.get(), t.perm.get(), ka.get(),
                           at.get(), kb.get(), hb.get(), vb.get(), cpos.get(), rc.get() + 1, n);
        SRF_HIP(hipGetLastError());
        // runs: numbers (exclusive scan of the starts) and first members
        const int32_t* md = rc.get() + 1;
        DevBuf<int32_t> rid(n + 1, st), rstart(n + 1, st);
        hipLaunchKernelGGL(k_run_starts, rgrid, dim3(B), 0, st, md, hb.get(), rid.get());
        SRF_HIP(hipGetLastError());
        exclusive_scan_i32_counted(rid.get(), n, md, st);
        hipLaunchKernelGGL(k_run_index, rgrid, dim3(B), 0, st, md, hb.get(), rid.get(),
                           rstart.get());
        SRF_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_run_rank, grid, dim3(B), 0, st, n, md, kb.get(), vb.get(), cpos.get(), rid.get(),
                           rstart.get(), t.perm.get(), d_flag);
        SRF_HIP(hipGetLastError());
    }
    t.px.alloc(n, st);
    t.py.alloc(n, st);
    t.pz.alloc(n, st);
    t.pm.alloc(n, st);
    t.release_events();
    if (full) {
        hipLaunchKernelGGL(k_gather<true>, dim3(grid_for(n, B, 1 << 30)), dim3(B), 0, st, n, t.perm.get(), x, y, z,
                           ps, m, ms, t.px.get(), t.py.get(), t.pz.get(), t.pm.get(), t.keys.get());
        SRF_HIP(hipGetLastError());
        return;
    }
    // the keys from the sort's words (ha sorted, ka still in input order);
    // the positions and masses on the second stream, where they overlap the
    // cell levels and the tree build's one synchronisation
    hipLaunchKernelGGL(k_sorted_keys, dim3(grid_for(n, B, 1 << 30)), dim3(B), 0, st, n, t.perm.get(), ha.get(),
                       ka.get(), t.keys.get());
    SRF_HIP(hipGetLastError());
    hipStream_t aux = aux_stream();
    SRF_HIP(hipEventCreateWithFlags(&t.sorted, hipEventDisableTiming));
    SRF_HIP(hipEventCreateWithFlags(&t.gathered, hipEventDisableTiming));
    SRF_HIP(hipEventRecord(t.sorted, st));
    SRF_HIP(hipStreamWaitEvent(aux, t.sorted, 0));
    hipLaunchKernelGGL(k_gather<false>, dim3(grid_for(n, B, 1 << 30)), dim3(B), 0, aux, n, t.perm.get(), x, y, z,
                       ps, m, ms, t.px.get(), t.py.get(), t.pz.get(), t.pm.get(), (uint64_t*)nullptr);
    SRF_HIP(hipGetLastError());
    SRF_HIP(hipEventRecord(t.gathered, aux));
}

}  // namespace srf
