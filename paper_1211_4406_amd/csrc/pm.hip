// Long-range (PM) half of the TreePM force split on one GPU (Sec. 2 split,
// PM steps of Sec. 2.2, "Relay Mesh Method"), in FP64 on a periodic n^3 mesh with points at
// x = i/n:
//   1. TSC assignment of the sorted particles to 27 mesh points each,
//   2. 3-D FFT (radix-2 Stockham, one pass per axis, lines staged in LDS),
//   3. multiplication by the Green's function
//        -4 pi G S(k)^2 / (k^2 W(k)^2),  S(k) = 12 (2 - 2 cos u - u sin u)/u^4,
//        u = |k| r_cut / 2 (the S2 cloud of the split),
//        W(k) = prod_axes sinc(k_a / 2n)^3 (the TSC window, deconvolved for
//        assignment and interpolation), zero at k = 0,
//   4. inverse FFT, 5. accelerations on the mesh by fourth-order central
//   differences, 6. TSC interpolation back to the particles.
#include <cmath>

#include "common.h"

namespace srf {
namespace {

// TSC stencil along one axis: nearest mesh point i0 = floor(u + 1/2) and
// weights of i0-1, i0, i0+1 for u = x n.
struct Tsc {
    int i[3];
    double w[3];
};

__device__ __forceinline__ Tsc tsc(double x, int n) {
    const double u = x * n;
    const double c = floor(u + 0.5);
    const double d = u - c;
    Tsc t;
    const int i0 = (int)c;
    t.i[0] = (i0 - 1 + n) % n;
    t.i[1] = i0 % n;
    t.i[2] = (i0 + 1) % n;
    t.w[0] = 0.5 * (0.5 - d) * (0.5 - d);
    t.w[1] = 0.75 - d * d;
    t.w[2] = 0.5 * (0.5 + d) * (0.5 + d);
    return t;
}

// 1. density (mass per unit volume) into the real parts of the complex mesh.
// A workgroup takes kChunk consecutive sorted particles, which lie close
// together (Morton order).  It finds the box of mesh points their stencils
// touch; if that box fits kBoxMax points, the 27 contributions of each
// particle are summed into the box in LDS and the box is then added to the
// mesh with one global atomic per touched point; otherwise each
// contribution goes to the mesh directly.
constexpr int kAssignThreads = 256;
constexpr int kChunk = 2048;
constexpr int kBoxMax = 4096;   // FP64 values in LDS (32 KB)

__device__ __forceinline__ int wrap_i(int i, int n) { return ((i % n) + n) % n; }

__global__ __launch_bounds__(kAssignThreads) void k_tsc_assign(int64_t np, const double* __restrict__ px,
                                                               const double* __restrict__ py,
                                                               const double* __restrict__ pz,
                                                               const double* __restrict__ pm, int n,
                                                               double* __restrict__ mesh) {
    __shared__ double box[kBoxMax];
    __shared__ int red[6][kAssignThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * kChunk;
    const int cnt = (int)((np - s0) < kChunk ? (np - s0) : kChunk);
    const double q = (double)n * n * n;
    // unwrapped nearest mesh points of this chunk: bounding box
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int k = tid; k < cnt; k += kAssignThreads) {
        const double u[3] = {px[s0 + k] * n, py[s0 + k] * n, pz[s0 + k] * n};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int c = (int)floor(u[a] + 0.5);
            lo[a] = min(lo[a], c);
            hi[a] = max(hi[a], c);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int o = 32; o >= 1; o >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = max(hi[a], __shfl_xor(hi[a], o, 64));
        }
        if (lane == 0) {
            red[a][wid] = lo[a];
            red[3 + a][wid] = hi[a];
        }
    }
    __syncthreads();
    int b0[3], bd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int l = red[a][0], h = red[3 + a][0];
        for (int w = 1; w < kAssignThreads / 64; ++w) {
            l = min(l, red[a][w]);
            h = max(h, red[3 + a][w]);
        }
        b0[a] = l - 1;
        bd[a] = h - l + 3;
    }
    const int64_t vol = (int64_t)bd[0] * bd[1] * bd[2];
    const int64_t nn = n;
    if (vol <= kBoxMax && bd[0] <= n && bd[1] <= n && bd[2] <= n) {
        for (int k = tid; k < vol; k += kAssignThreads) box[k] = 0.0;
        __syncthreads();
        for (int k = tid; k < cnt; k += kAssignThreads) {
            const int64_t s = s0 + k;
            const double u[3] = {px[s] * n, py[s] * n, pz[s] * n};
            int c[3];
            double w[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ci = floor(u[a] + 0.5);
                const double d = u[a] - ci;
                c[a] = (int)ci - b0[a];   // stencil centre, box-relative (>= 1)
                w[a][0] = 0.5 * (0.5 - d) * (0.5 - d);
                w[a][1] = 0.75 - d * d;
                w[a][2] = 0.5 * (0.5 + d) * (0.5 + d);
            }
            const double mq = pm[s] * q;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double wij = mq * w[0][i] * w[1][j];
                    const int row = ((c[0] - 1 + i) * bd[1] + (c[1] - 1 + j)) * bd[2] + c[2] - 1;
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) atomicAdd(&box[row + kk], wij * w[2][kk]);
                }
        }
        __syncthreads();
        for (int k = tid; k < vol; k += kAssignThreads) {
            const double v = box[k];
            if (v == 0.0) continue;
            const int iz = k % bd[2], iy = (k / bd[2]) % bd[1], ix = k / (bd[2] * bd[1]);
            const int64_t g = ((int64_t)wrap_i(b0[0] + ix, n) * nn + wrap_i(b0[1] + iy, n)) * nn + wrap_i(b0[2] + iz, n);
            unsafeAtomicAdd(mesh + 2 * g, v);
        }
        return;
    }
    for (int k = tid; k < cnt; k += kAssignThreads) {
        const int64_t s = s0 + k;
        const Tsc a = tsc(px[s], n), b = tsc(py[s], n), c = tsc(pz[s], n);
        const double mq = pm[s] * q;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double wij = mq * a.w[i] * b.w[j];
                const int64_t row = ((int64_t)a.i[i] * nn + b.i[j]) * nn;
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) unsafeAtomicAdd(mesh + 2 * (row + c.i[kk]), wij * c.w[kk]);
            }
    }
}

// twiddles exp(-2 pi i j / n), j < n/2
__global__ void k_twiddle(int n, double2* __restrict__ tw) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n / 2) return;
    double s, c;
    sincospi(-2.0 * j / n, &s, &c);
    tw[j] = make_double2(c, s);
}

// 2. and 4. One FFT pass: length-n transforms of all n^2 lines along one
// axis.  A workgroup stages kBn / n lines in LDS (consecutive in the
// contiguous mesh index, so that loads and stores are coalesced), runs the
// log2(n) radix-2 Stockham stages there, and writes back in place.
// axis 2 (contiguous): line L starts at L n, element stride 1;
// axis 1: line L = (x, z) starts at x n^2 + z, stride n;
// axis 0: line L = (y, z) starts at L, stride n^2.
constexpr int kFftThreads = 256;
constexpr int kBn = 2048;   // complex values staged per workgroup

template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft_axis(double2* __restrict__ mesh, int n, int log2n, int axis,
                                                           const double2* __restrict__ tw) {
    __shared__ double2 bufA[kBn];
    __shared__ double2 bufB[kBn];
    const int B = kBn / n;                    // lines per workgroup
    const int64_t nn = n;
    const int64_t L0 = (int64_t)blockIdx.x * B;
    const int64_t es = axis == 2 ? 1 : (axis == 1 ? nn : nn * nn);
    auto base = [&](int64_t L) -> int64_t {
        return axis == 2 ? L * nn : (axis == 1 ? (L / nn) * nn * nn + (L % nn) : L);
    };
    // load: line-major in LDS (line b occupies [b n, b n + n))
    for (int idx = threadIdx.x; idx < kBn; idx += kFftThreads) {
        int b, j;
        if (axis == 2) {
            b = idx / n;
            j = idx % n;
        } else {
            j = idx / B;
            b = idx % B;
        }
        bufA[b * n + j] = mesh[base(L0 + b) + j * es];
    }
    __syncthreads();
    double2* in = bufA;
    double2* out = bufB;
    const int half = n / 2;
    for (int st = 0, m = 1; st < log2n; ++st, m <<= 1) {
        for (int t = threadIdx.x; t < kBn / 2; t += kFftThreads) {
            const int b = t / half, q = t % half;
            const int k = q & (m - 1);
            double2 w = tw[k * (half / m)];
            if (INV) w.y = -w.y;
            const double2 u = in[b * n + q], v0 = in[b * n + q + half];
            const double2 v = make_double2(v0.x * w.x - v0.y * w.y, v0.x * w.y + v0.y * w.x);
            out[b * n + 2 * q - k] = make_double2(u.x + v.x, u.y + v.y);
            out[b * n + 2 * q - k + m] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
        double2* tmp = in;
        in = out;
        out = tmp;
    }
    for (int idx = threadIdx.x; idx < kBn; idx += kFftThreads) {
        int b, j;
        if (axis == 2) {
            b = idx / n;
            j = idx % n;
        } else {
            j = idx / B;
            b = idx % B;
        }
        mesh[base(L0 + b) + j * es] = in[b * n + j];
    }
}

__device__ __forceinline__ double wavenumber(int i, int n) {
    return 2.0 * M_PI * (double)(i < n / 2 ? i : i - n);
}

__device__ __forceinline__ double sinc(double v) { return v == 0.0 ? 1.0 : sin(v) / v; }

// Transform of the unit-mass S2 cloud at u = k r_cut / 2; Taylor series
// below u = 1/2, where the closed form's O(1) terms cancel to O(u^4).
__device__ __forceinline__ double s2_shape(double u) {
    if (u < 0.5) {
        const double v = u * u;
        return 1.0 + v * (-1.0 / 15.0 + v * (1.0 / 560.0 + v * (-1.0 / 37800.0 + v / 3991680.0)));
    }
    double s, c;
    sincos(u, &s, &c);
    return 12.0 * (2.0 - 2.0 * c - u * s) / (u * u * u * u);
}

// 3. spectrum *= Green's function / n^3 (the inverse FFT is unnormalised)
__global__ void k_green(double2* __restrict__ mesh, int n, double r_cut, double G) {
    const int64_t nn = n;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= nn * nn * nn) return;
    const int iz = (int)(idx % nn), iy = (int)((idx / nn) % nn), ix = (int)(idx / (nn * nn));
    if (idx == 0) {
        mesh[0] = make_double2(0.0, 0.0);
        return;
    }
    const double kx = wavenumber(ix, n), ky = wavenumber(iy, n), kz = wavenumber(iz, n);
    const double k2 = kx * kx + ky * ky + kz * kz;
    const double h = 0.5 / n;
    const double w1 = sinc(kx * h) * sinc(ky * h) * sinc(kz * h);
    const double W = w1 * w1 * w1;
    const double S = s2_shape(sqrt(k2) * r_cut * 0.5);
    const double g = -4.0 * M_PI * G * S * S / (k2 * W * W) / ((double)n * n * n);
    const double2 v = mesh[idx];
    mesh[idx] = make_double2(v.x * g, v.y * g);
}

// 5. a = -grad phi, fourth-order central differences, from the real parts;
// the three components of a mesh point side by side (x, y, z, unused), so
// that the interpolation reads one 32-byte record per stencil point
__global__ void k_fd4(const double2* __restrict__ phi, int n, double4* __restrict__ acc) {
    const int64_t nn = n;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= nn * nn * nn) return;
    const int iz = (int)(idx % nn), iy = (int)((idx / nn) % nn), ix = (int)(idx / (nn * nn));
    auto at = [&](int x, int y, int z) -> double {
        x = (x + n) % n;
        y = (y + n) % n;
        z = (z + n) % n;
        return phi[((int64_t)x * nn + y) * nn + z].x;
    };
    const double c1 = 2.0 / 3.0 * n, c2 = 1.0 / 12.0 * n;
    double4 a;
    a.x = -(c1 * (at(ix + 1, iy, iz) - at(ix - 1, iy, iz)) - c2 * (at(ix + 2, iy, iz) - at(ix - 2, iy, iz)));
    a.y = -(c1 * (at(ix, iy + 1, iz) - at(ix, iy - 1, iz)) - c2 * (at(ix, iy + 2, iz) - at(ix, iy - 2, iz)));
    a.z = -(c1 * (at(ix, iy, iz + 1) - at(ix, iy, iz - 1)) - c2 * (at(ix, iy, iz + 2) - at(ix, iy, iz - 2)));
    a.w = 0.0;
    acc[idx] = a;
}

// 6. TSC interpolation at the sorted particles; output in input order
__global__ void k_tsc_interp(int64_t np, const double* __restrict__ px, const double* __restrict__ py,
                             const double* __restrict__ pz, const int32_t* __restrict__ perm, int n,
                             const double4* __restrict__ acc, double* __restrict__ ax, double* __restrict__ ay,
                             double* __restrict__ az, int64_t os) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= np) return;
    const Tsc a = tsc(px[s], n), b = tsc(py[s], n), c = tsc(pz[s], n);
    const int64_t nn = n;
    double fx = 0, fy = 0, fz = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double wij = a.w[i] * b.w[j];
            const int64_t row = ((int64_t)a.i[i] * nn + b.i[j]) * nn;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double w = wij * c.w[k];
                const double4 m = acc[row + c.i[k]];
                fx += w * m.x;
                fy += w * m.y;
                fz += w * m.z;
            }
        }
    const int64_t o = (int64_t)perm[s] * os;
    ax[o] = fx;
    ay[o] = fy;
    az[o] = fz;
}

void fft3(double2* mesh, int n, const double2* tw, bool inv, hipStream_t st) {
    int log2n = 0;
    while ((1 << log2n) < n) ++log2n;
    const unsigned blocks = (unsigned)((int64_t)n * n / (kBn / n));
    for (int axis = 2; axis >= 0; --axis) {
        if (inv)
            hipLaunchKernelGGL(k_fft_axis<true>, dim3(blocks), dim3(kFftThreads), 0, st, mesh, n, log2n, axis, tw);
        else
            hipLaunchKernelGGL(k_fft_axis<false>, dim3(blocks), dim3(kFftThreads), 0, st, mesh, n, log2n, axis, tw);
        SRF_HIP(hipGetLastError());
    }
}

}  // namespace

void launch_pm(const Tree& t, double G, double r_cut, int n, double* ax, double* ay, double* az, int64_t os,
               hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const int64_t np = t.n;
    const int64_t cells = (int64_t)n * n * n;
    DevBuf<double2> mesh(cells, st);
    DevBuf<double2> tw(n / 2, st);
    DevBuf<double4> acc(cells, st);
    if (ev0) SRF_HIP(hipEventRecord(ev0, st));
    fill_f64(reinterpret_cast<double*>(mesh.get()), 0.0, 2 * cells, st);
    hipLaunchKernelGGL(k_twiddle, dim3((unsigned)((n / 2 + 255) / 256)), dim3(256), 0, st, n, tw.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tsc_assign, dim3((unsigned)((np + kChunk - 1) / kChunk)), dim3(kAssignThreads), 0, st, np,
                       t.px.get(), t.py.get(), t.pz.get(), t.pm.get(), n, reinterpret_cast<double*>(mesh.get()));
    SRF_HIP(hipGetLastError());
    fft3(mesh.get(), n, tw.get(), false, st);
    hipLaunchKernelGGL(k_green, dim3(grid_for(cells, 256, 1 << 30)), dim3(256), 0, st, mesh.get(), n, r_cut, G);
    SRF_HIP(hipGetLastError());
    fft3(mesh.get(), n, tw.get(), true, st);
    hipLaunchKernelGGL(k_fd4, dim3(grid_for(cells, 256, 1 << 30)), dim3(256), 0, st, mesh.get(), n, acc.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tsc_interp, dim3(grid_for(np, 256, 1 << 30)), dim3(256), 0, st, np, t.px.get(), t.py.get(),
                       t.pz.get(), t.perm.get(), n, acc.get(), ax, ay, az, os);
    SRF_HIP(hipGetLastError());
    if (ev1) SRF_HIP(hipEventRecord(ev1, st));
}

}  // namespace srf
