// Kick and drift of the multiple-stepsize integrator (Sec. 3: one step is
// one PM cycle and two PP cycles): v += a dt and x += v dt with x wrapped
// into the periodic unit box.
#include "common.h"

namespace srf {
namespace {

__global__ void k_kick(int64_t n, double* __restrict__ vx, double* __restrict__ vy, double* __restrict__ vz,
                       int64_t vs, const double* __restrict__ ax, const double* __restrict__ ay,
                       const double* __restrict__ az, int64_t as, double dt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    vx[i * vs] += dt * ax[i * as];
    vy[i * vs] += dt * ay[i * as];
    vz[i * vs] += dt * az[i * as];
}

__device__ __forceinline__ double wrap_unit(double v) {
    const double u = v - floor(v);
    return u >= 1.0 ? 0.0 : u;
}

__global__ void k_drift(int64_t n, double* __restrict__ x, double* __restrict__ y, double* __restrict__ z,
                        int64_t xs, const double* __restrict__ vx, const double* __restrict__ vy,
                        const double* __restrict__ vz, int64_t vs, double dt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i * xs] = wrap_unit(x[i * xs] + dt * vx[i * vs]);
    y[i * xs] = wrap_unit(y[i * xs] + dt * vy[i * vs]);
    z[i * xs] = wrap_unit(z[i * xs] + dt * vz[i * vs]);
}

}  // namespace

void launch_kick(int64_t n, double* vx, double* vy, double* vz, int64_t vs, const double* ax, const double* ay,
                 const double* az, int64_t as, double dt, hipStream_t st) {
    hipLaunchKernelGGL(k_kick, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, n, vx, vy, vz, vs, ax, ay, az, as,
                       dt);
    SRF_HIP(hipGetLastError());
}

void launch_drift(int64_t n, double* x, double* y, double* z, int64_t xs, const double* vx, const double* vy,
                  const double* vz, int64_t vs, double dt, hipStream_t st) {
    hipLaunchKernelGGL(k_drift, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, n, x, y, z, xs, vx, vy, vz, vs,
                       dt);
    SRF_HIP(hipGetLastError());
}

}  // namespace srf
