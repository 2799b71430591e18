// Steps a1-a2: periodic wrap, 63-bit Morton keys, stable LSD radix sort of
// (key, input index), gather of the sorted SoA particle arrays.
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
                       uint64_t* __restrict__ keys, int32_t* __restrict__ vals, int32_t* __restrict__ flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a = x[i * ps], b = y[i * ps], c = z[i * ps], mm = m[i * ms];
    int bad = 0;
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) bad |= 1;
    if (!(isfinite(mm) && mm > 0.0)) bad |= 2;
    if (bad) atomicOr(flag, bad);
    uint64_t kx = grid21(wrap01(a)), ky = grid21(wrap01(b)), kz = grid21(wrap01(c));
    keys[i] = (spread3(kx) << 2) | (spread3(ky) << 1) | spread3(kz);
    vals[i] = (int32_t)i;
}

// ------------------------------------------------------------- radix sort
constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // keys per block
constexpr int kDigits = 256;

__global__ __launch_bounds__(kThreads) void k_hist(int64_t n, const uint64_t* __restrict__ keys, int shift,
                                                   int64_t tiles, int32_t* __restrict__ counts) {
    __shared__ int32_t h[kDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = blockIdx.x * (int64_t)kTile;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + k * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter.  The keys of a tile are taken in rounds of 256 (position
// round*256 + tid); a key's rank among equal digits is the count of that
// digit in earlier rounds plus the count among lower threads this round.
// The tile is then reordered by digit in LDS, so that the global writes of
// each digit's run are contiguous.
__global__ __launch_bounds__(kThreads) void k_scatter(int64_t n, const uint64_t* __restrict__ kin,
                                                      const int32_t* __restrict__ vin, uint64_t* __restrict__ kout,
                                                      int32_t* __restrict__ vout, int shift, int64_t tiles,
                                                      const int32_t* __restrict__ offsets) {
    __shared__ int32_t base[kDigits];
    __shared__ int32_t run[kDigits];
    __shared__ int32_t toff[kDigits];
    __shared__ int32_t wc[kThreads / 64][kDigits];
    __shared__ uint64_t skey[kTile];
    __shared__ int32_t sval[kTile];
    __shared__ int32_t wsum[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    base[tid] = offsets[(int64_t)tid * tiles + blockIdx.x];
    run[tid] = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) wc[w][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tbase = blockIdx.x * (int64_t)kTile;
    uint64_t key[kItems];
    int32_t val[kItems], dig[kItems], rank[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = tbase + r * kThreads + tid;
        const bool valid = i < n;
        key[r] = valid ? kin[i] : 0;
        val[r] = valid ? vin[i] : 0;
        const int d = valid ? (int)((key[r] >> shift) & 0xff) : -1;
        dig[r] = d;
        // lanes holding the same digit (invalid lanes match nobody valid)
        uint64_t peers = __ballot(valid);
        if (!valid) peers = ~peers;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = valid && ((d >> b) & 1);
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const int lower = __popcll(peers & lt);
        if (valid && lower == 0) wc[wid][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int rk = run[d] + lower;
            for (int w = 0; w < wid; ++w) rk += wc[w][d];
            rank[r] = rk;
        } else {
            rank[r] = 0;
        }
        __syncthreads();
        int tot = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            tot += wc[w][tid];
            wc[w][tid] = 0;
        }
        run[tid] += tot;
        __syncthreads();
    }
    // exclusive scan of the tile's digit counts (one digit per thread)
    {
        const int v = run[tid];
        int incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        int off = incl - v;
        for (int w = 0; w < wid; ++w) off += wsum[w];
        toff[tid] = off;
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        if (dig[r] < 0) continue;
        const int p = toff[dig[r]] + rank[r];
        skey[p] = key[r];
        sval[p] = val[r];
    }
    __syncthreads();
    const int cnt = (int)((n - tbase) < kTile ? (n - tbase) : kTile);
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int p = r * kThreads + tid;
        if (p < cnt) {
            const uint64_t k = skey[p];
            const int d = (int)((k >> shift) & 0xff);
            const int64_t dst = (int64_t)base[d] + (p - toff[d]);
            kout[dst] = k;
            vout[dst] = sval[p];
        }
    }
}

__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ x,
                         const double* __restrict__ y, const double* __restrict__ z, int64_t ps,
                         const double* __restrict__ m, int64_t ms, double* __restrict__ px, double* __restrict__ py,
                         double* __restrict__ pz, double* __restrict__ pm) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t i = perm[s];
    px[s] = wrap01(x[i * ps]);
    py[s] = wrap01(y[i * ps]);
    pz[s] = wrap01(z[i * ps]);
    pm[s] = m[i * ms];
}

}  // namespace

void build_sorted(Tree& t, const double* x, const double* y, const double* z, int64_t ps, const double* m,
                  int64_t ms, int32_t* d_flag, hipStream_t st) {
    const int64_t n = t.n;
    DevBuf<uint64_t> kb(n, st);
    DevBuf<int32_t> vb(n, st);
    t.keys.alloc(n, st);
    t.perm.alloc(n, st);
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, n, x, y, z, ps, m, ms,
                       t.keys.get(), t.perm.get(), d_flag);
    SRF_HIP(hipGetLastError());
    const int64_t tiles = (n + kTile - 1) / kTile;
    DevBuf<int32_t> counts(kDigits * tiles, st);
    uint64_t* ka = t.keys.get();
    int32_t* va = t.perm.get();
    uint64_t* kk = kb.get();
    int32_t* vv = vb.get();
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_hist, dim3((unsigned)tiles), dim3(kThreads), 0, st, n, ka, shift, tiles, counts.get());
        SRF_HIP(hipGetLastError());
        exclusive_scan_i32(counts.get(), kDigits * tiles, false, st);
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)tiles), dim3(kThreads), 0, st, n, ka, va, kk, vv, shift, tiles,
                           counts.get());
        SRF_HIP(hipGetLastError());
        std::swap(ka, kk);
        std::swap(va, vv);
    }
    // eight passes: the result is back in t.keys / t.perm
    t.px.alloc(n, st);
    t.py.alloc(n, st);
    t.pz.alloc(n, st);
    t.pm.alloc(n, st);
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, n, t.perm.get(), x, y, z, ps, m,
                       ms, t.px.get(), t.py.get(), t.pz.get(), t.pm.get());
    SRF_HIP(hipGetLastError());
}

}  // namespace srf
