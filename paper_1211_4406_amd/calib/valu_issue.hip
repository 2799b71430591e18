// Issue-rate calibration of the vector ALU (measurement tool, not part of
// the gravity library): how many cycles one SIMD spends per wave64
// instruction of a given kind, the unit that turns the pair kernels'
// instruction counts into time.
//
// Each kernel runs CH independent dependency chains per lane for `iters`
// rounds; every wave reads the shader clock (s_memtime) before and after
// its loop and stores the difference.  With W waves resident on each SIMD
// and every wave issuing CH * iters instructions of the measured kind,
//   cycles per instruction = elapsed cycles / (W * CH * iters)
// (the waves of a SIMD share its issue slots, so each wave's elapsed time
// covers the instructions of all W).  Loop control is scalar and overlaps.
//
// Kinds (all FP32 unless noted):
//   0  v_fma_f32, every operand in a vector register
//   1  v_fma_f32 with one scalar-register operand
//   2  v_rsq_f32
//   3  v_sqrt_f32
//   4  v_fma_f64, every operand in a vector register
//   5  v_fma_f32 with every operand in a vector register, 1 chain per lane
//      (latency bound: no independent work to interleave)
//   6  v_add_f32 with a DPP quad permutation of one operand
//   7  v_add_f32 with the DPP half-row mirror
//   8  v_add_f32 with the DPP row mirror
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kCh = 8;

__device__ __forceinline__ float vpin(float x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ double vpin(double x) {
    asm volatile("" : "+v"(x));
    return x;
}

template <int CTRL>
__device__ __forceinline__ float dpp_add(float a) {
    return a + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, a), CTRL, 0xf, 0xf,
                                                                     false));
}

template <int KIND>
__global__ __launch_bounds__(256) void k_issue(int iters, float sb, float* __restrict__ sink,
                                               uint64_t* __restrict__ cycles) {
    const int tid = threadIdx.x;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + tid) >> 6;
    float a[kCh];
    double d[kCh];
#pragma unroll
    for (int k = 0; k < kCh; ++k) {
        a[k] = vpin(1.0f + 1e-3f * (float)(k + tid));
        d[k] = vpin(1.0 + 1e-3 * (double)(k + tid));
    }
    const float b = vpin(0.999f), c = vpin(1e-4f);
    const double db = vpin(0.999), dc = vpin(1e-4);
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (KIND == 5) {
                a[0] = __builtin_fmaf(a[0], b, c);
                a[0] = __builtin_fmaf(a[0], b, c);
            } else {
#pragma unroll
                for (int k = 0; k < kCh; ++k) {
                    if (KIND == 0) a[k] = __builtin_fmaf(a[k], b, c);
                    if (KIND == 1) a[k] = __builtin_fmaf(a[k], sb, c);
                    if (KIND == 2) a[k] = __builtin_amdgcn_rsqf(a[k]);
                    if (KIND == 3) a[k] = __builtin_amdgcn_sqrtf(a[k]);
                    if (KIND == 4) d[k] = __builtin_fma(d[k], db, dc);
                    if (KIND >= 6) {
                        // the values double each step and saturate at inf, which costs nothing
                        a[k] = dpp_add<KIND == 6 ? 0xB1 : (KIND == 7 ? 0x141 : 0x140)>(a[k]);
                        asm volatile("" : "+v"(a[k]));   // keeps each add fused with its DPP read
                    }
                }
            }
        }
    }
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kCh; ++k) s += a[k] + (float)d[k];
    sink[blockIdx.x * (int64_t)blockDim.x + tid] = s;
    if ((tid & 63) == 0) cycles[wave] = t1 - t0;
}

// Instructions of the measured kind per wave per round of the loop.
int per_round(int kind) { return kind == 5 ? 8 : 4 * kCh; }

}  // namespace

extern "C" {

// Run kind `kind` with `waves_per_simd` waves on each SIMD of `n_cu` compute
// units for `iters` rounds.  Writes the median over waves of the elapsed
// shader cycles per instruction per SIMD (*cpi) and the kernel's wall time
// (*ms, HIP events).  Returns 0, or -1 for an invalid argument, -4 for a
// HIP error.
int srf_calib_valu(int kind, int n_cu, int waves_per_simd, int iters, double* cpi, double* ms) {
    if (kind < 0 || kind > 8 || n_cu < 1 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !cpi || !ms)
        return -1;
    const int64_t blocks = (int64_t)n_cu * waves_per_simd;   // 4 waves per block: one per SIMD
    const int64_t threads = blocks * 256, waves = threads / 64;
    float* sink = nullptr;
    uint64_t* cyc = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipMalloc(&sink, threads * sizeof(float)) != hipSuccess) return -4;
    if (hipMalloc(&cyc, waves * sizeof(uint64_t)) != hipSuccess) {
        (void)hipFree(sink);
        return -4;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -4;
    if (rc == 0) {
        (void)hipEventRecord(e0, nullptr);
        switch (kind) {
            case 0: hipLaunchKernelGGL(k_issue<0>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            case 1: hipLaunchKernelGGL(k_issue<1>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            case 2: hipLaunchKernelGGL(k_issue<2>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            case 3: hipLaunchKernelGGL(k_issue<3>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            case 4: hipLaunchKernelGGL(k_issue<4>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            case 5: hipLaunchKernelGGL(k_issue<5>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            case 6: hipLaunchKernelGGL(k_issue<6>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            case 7: hipLaunchKernelGGL(k_issue<7>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
            default: hipLaunchKernelGGL(k_issue<8>, dim3((unsigned)blocks), dim3(256), 0, nullptr, iters, 0.999f, sink, cyc); break;
        }
        if (hipGetLastError() != hipSuccess) rc = -4;
        (void)hipEventRecord(e1, nullptr);
        if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -4;
    }
    if (rc == 0) {
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t;
        uint64_t* h = new uint64_t[waves];
        if (hipMemcpy(h, cyc, waves * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess) rc = -4;
        if (rc == 0) {
            // median by partial selection
            int64_t lo = 0, hi = waves - 1, k = waves / 2;
            while (lo < hi) {
                const uint64_t piv = h[(lo + hi) / 2];
                int64_t i = lo, j = hi;
                while (i <= j) {
                    while (h[i] < piv) ++i;
                    while (h[j] > piv) --j;
                    if (i <= j) {
                        const uint64_t tmp = h[i];
                        h[i] = h[j];
                        h[j] = tmp;
                        ++i;
                        --j;
                    }
                }
                if (k <= j) hi = j;
                else if (k >= i) lo = i;
                else break;
            }
            *cpi = (double)h[k] / ((double)waves_per_simd * per_round(kind) * iters);
        }
        delete[] h;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipFree(cyc);
    return rc;
}

}  // extern "C"
