// Quadrupole term of the accepted cells (accuracy variant of the cell
// expansion of Sec. 1, taken one order past the monopole).
//
// A cell of second moments S = sum_k m_k (x_k - X)(x_k - X)^T about its
// centre of mass X adds, to the pull M F(D) of its monopole on a target at
// offset D = X - x (F(D) = D phi(|D|), phi = g(k r) / s^3, k = 2 / r_cut,
// s^2 = r^2 + eps^2),
//   1/2 S_ab d_a d_b F(D) = psi S D + (psi tr(S) / 2 + chi (D . S D) / 2) D
// with psi = phi'(r) / r and chi = psi'(r) / r:
//   psi = s^-3 (h - 3 s^-2 g),  chi = s^-3 (j - s^-2 (6 h - 15 s^-2 g)),
//   h = k^2 H(xi),  j = k^4 H'(xi) / xi,  H = g'(xi) / xi.
// On [0, 1]  g = 1 - 8/5 xi^3 + 8/5 xi^5 - 1/2 xi^6 - 12/35 xi^7 + 3/20 xi^8,
//            H = -24/5 xi + 8 xi^3 - 3 xi^4 - 12/5 xi^5 + 6/5 xi^6,
//            H'/xi = -24/5 / xi + 24 xi - 12 xi^2 - 12 xi^3 + 36/5 xi^4;
// on [1, 2]  (t = 2 - xi)  g = t^5 (7 xi^3 + 22 xi^2 + 10 xi + 4) / 140,
//            H = -t^4 (2 xi^2 + 4 xi - 1) / 5,  H'/xi = 12/5 t^3 (xi + 1 - 1/xi);
// every form is written in r with the powers of k folded into the
// coefficients, and 0 at and beyond r_cut through the clamp of t.
//
// Three kernels: mark the cells that occur in some list, their second
// moments (FP64, 64 cells per wave), and the correction pass (one wave per
// group, targets in lanes, the list's cells compacted into LDS in chunks of
// 256 entries, split near/far as in the force kernel), which adds G times
// the term to the accelerations.
#include "common.h"

namespace srf {
namespace {

template <class T>
struct QCoef {
    T A3, A5, A6, A7, A8;          // g on [0,1] - 1, in r
    T B1, B3, B4, B5, B6;          // k^2 H on [0,1], in r
    T J0, J1, J2, J3, J4;          // k^4 H'/xi on [0,1]: J0 / r + r (J1 + ...)
    T C0, C1, C2, C3;              // g on [1,2] / t^5
    T E0, E1, E2;                  // -k^2 H on [1,2] / t^4
    T F0, F1, F2;                  // k^4 H'/xi on [1,2] / t^3: F0 / r + F1 + F2 r
    T k, eps2, rh2;
    T three, six, fifteen;         // held in registers (not inline constants)
};

template <class T>
QCoef<T> make_qcoef(double rc, double eps) {
    const double k = 2.0 / rc, k2 = k * k, k3 = k2 * k, k4 = k3 * k, k5 = k4 * k, k6 = k5 * k, k7 = k6 * k,
                 k8 = k7 * k;
    QCoef<T> c;
    c.A3 = (T)(-8.0 / 5.0 * k3);
    c.A5 = (T)(8.0 / 5.0 * k5);
    c.A6 = (T)(-0.5 * k6);
    c.A7 = (T)(-12.0 / 35.0 * k7);
    c.A8 = (T)(3.0 / 20.0 * k8);
    c.B1 = (T)(-24.0 / 5.0 * k3);
    c.B3 = (T)(8.0 * k5);
    c.B4 = (T)(-3.0 * k6);
    c.B5 = (T)(-12.0 / 5.0 * k7);
    c.B6 = (T)(6.0 / 5.0 * k8);
    c.J0 = (T)(-24.0 / 5.0 * k3);
    c.J1 = (T)(24.0 * k5);
    c.J2 = (T)(-12.0 * k6);
    c.J3 = (T)(-12.0 * k7);
    c.J4 = (T)(36.0 / 5.0 * k8);
    c.C0 = (T)(4.0 / 140.0);
    c.C1 = (T)(10.0 / 140.0 * k);
    c.C2 = (T)(22.0 / 140.0 * k2);
    c.C3 = (T)(7.0 / 140.0 * k3);
    c.E0 = (T)(-k2 / 5.0);
    c.E1 = (T)(4.0 / 5.0 * k3);
    c.E2 = (T)(2.0 / 5.0 * k4);
    c.F0 = (T)(-12.0 / 5.0 * k3);
    c.F1 = (T)(12.0 / 5.0 * k4);
    c.F2 = (T)(12.0 / 5.0 * k5);
    c.k = (T)k;
    c.eps2 = (T)(eps * eps);
    c.rh2 = (T)(0.25 * rc * rc);
    c.three = (T)3;
    c.six = (T)6;
    c.fifteen = (T)15;
    return c;
}

__device__ __forceinline__ float q_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double q_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float q_sat(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }
__device__ __forceinline__ double q_sat(double x) { return fmin(fmax(x, 0.0), 1.0); }

// Keep a loop-invariant value in a vector register (the empty asm makes it
// opaque), so that the pair arithmetic reads VGPR operands only.
__device__ __forceinline__ float q_pin(float x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ double q_pin(double x) {
    asm volatile("" : "+v"(x));
    return x;
}

template <class T>
__device__ __forceinline__ QCoef<T> q_pinned(const QCoef<T>& a) {
    QCoef<T> c;
    c.A3 = q_pin(a.A3); c.A5 = q_pin(a.A5); c.A6 = q_pin(a.A6); c.A7 = q_pin(a.A7); c.A8 = q_pin(a.A8);
    c.B1 = q_pin(a.B1); c.B3 = q_pin(a.B3); c.B4 = q_pin(a.B4); c.B5 = q_pin(a.B5); c.B6 = q_pin(a.B6);
    c.J0 = q_pin(a.J0); c.J1 = q_pin(a.J1); c.J2 = q_pin(a.J2); c.J3 = q_pin(a.J3); c.J4 = q_pin(a.J4);
    c.C0 = q_pin(a.C0); c.C1 = q_pin(a.C1); c.C2 = q_pin(a.C2); c.C3 = q_pin(a.C3);
    c.E0 = q_pin(a.E0); c.E1 = q_pin(a.E1); c.E2 = q_pin(a.E2);
    c.F0 = q_pin(a.F0); c.F1 = q_pin(a.F1); c.F2 = q_pin(a.F2);
    c.k = q_pin(a.k); c.eps2 = q_pin(a.eps2); c.rh2 = q_pin(a.rh2);
    c.three = q_pin(a.three); c.six = q_pin(a.six); c.fifteen = q_pin(a.fifteen);
    return c;
}

template <class T>
struct QV4 {};
template <>
struct QV4<float> { using type = float4; };
template <>
struct QV4<double> { using type = double4; };
template <class T>
struct QV2 {};
template <>
struct QV2<float> { using type = float2; };
template <>
struct QV2<double> { using type = double2; };

// Cells that occur as an entry of some list (flags set to 1; the buffer is
// cleared before).
__global__ void k_mark_cells(int64_t n_entries, const int32_t* __restrict__ ent, int32_t* __restrict__ used) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_entries;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = ent[e];
        if (v < 0) used[-(int64_t)v - 1] = 1;
    }
}

// S_c = sum_k m_k (x_k - X_c)(x_k - X_c)^T as (xx, yy, zz, xy, xz, yz) for
// the marked cells.  One wave takes 64 consecutive cells: a cell of at most
// kSmallCell particles is summed by its own lane; each larger one is summed
// by the whole wave (lanes stride over its particles, partial sums combined
// in a fixed order).  Deterministic either way.  Offsets x_k - X_c are taken
// to the nearest periodic image (a refitted cell may straddle a face of the
// unit box; the root, never a source, is not computed).
constexpr int32_t kSmallCell = 64;

__device__ __forceinline__ void add_second(double (&a)[6], double m, double dx, double dy, double dz) {
    a[0] += m * dx * dx;
    a[1] += m * dy * dy;
    a[2] += m * dz * dz;
    a[3] += m * dx * dy;
    a[4] += m * dx * dz;
    a[5] += m * dy * dz;
}

__global__ __launch_bounds__(64) void k_second_moments(int64_t nn, const NodeRange* __restrict__ range,
                                                       const int32_t* __restrict__ used,
                                                       const double* __restrict__ px, const double* __restrict__ py,
                                                       const double* __restrict__ pz, const double* __restrict__ pm,
                                                       const double* __restrict__ nX, const double* __restrict__ nY,
                                                       const double* __restrict__ nZ, double* __restrict__ S) {
    const int lane = threadIdx.x;
    const int64_t c = blockIdx.x * 64ll + lane;
    const bool on = c < nn && used[c];
    NodeRange rg;
    rg.first = rg.count = 0;
    double X = 0, Y = 0, Z = 0;
    if (on) {
        rg = range[c];
        X = nX[c];
        Y = nY[c];
        Z = nZ[c];
    }
    // small cells: one lane each
    if (on && rg.count <= kSmallCell) {
        double a[6] = {0, 0, 0, 0, 0, 0};
        for (int32_t k = rg.first; k < rg.first + rg.count; ++k) add_second(a, pm[k], image(px[k] - X), image(py[k] - Y), image(pz[k] - Z));
#pragma unroll
        for (int q = 0; q < 6; ++q) S[c * 6 + q] = a[q];
    }
    // large cells: the whole wave, one after another
    uint64_t big = __ballot(on && rg.count > kSmallCell);
    while (big) {
        const int l = __ffsll((unsigned long long)big) - 1;
        big &= big - 1;
        const int32_t f = __shfl(rg.first, l, 64), n = __shfl(rg.count, l, 64);
        const double bx = __shfl(X, l, 64), by = __shfl(Y, l, 64), bz = __shfl(Z, l, 64);
        double a[6] = {0, 0, 0, 0, 0, 0};
        for (int32_t k = f + lane; k < f + n; k += 64) add_second(a, pm[k], image(px[k] - bx), image(py[k] - by), image(pz[k] - bz));
#pragma unroll
        for (int q = 0; q < 6; ++q) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) a[q] += __shfl_xor(a[q], o, 64);
        }
        if (lane == l) {
#pragma unroll
            for (int q = 0; q < 6; ++q) S[c * 6 + q] = a[q];
        }
    }
}

// Term of one cell (offset p.xyz from the group centre, p.w = tr(S) / 2,
// s1 = (xx, yy, zz, xy), s2 = (xz, yz)) on the target at (xi, yi, zi).
// Without NEAR the cell lies at xi >= 1 from every target of the group and
// only the [1, 2] forms are evaluated.
template <class T, class V4, class V2, bool NEAR>
__device__ __forceinline__ void quad_pair(const V4& p, const V4& s1, const V2& s2, T xi, T yi, T zi,
                                          const QCoef<T>& c, T& ox, T& oy, T& oz) {
    const T dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
    const T r2 = dz * dz + dy * dy + dx * dx;
    const T rinv = q_rsqrt(r2 + c.eps2);
    const T u = rinv * rinv;
    const T ir = r2 > T(0) ? q_rsqrt(r2) : T(0);   // 1 / r (an accepted cell is never at r = 0)
    const T r = r2 * ir;
    // [1, 2] forms
    const T t = q_sat(T(2) - c.k * r);
    const T t2 = t * t, t3 = t2 * t, t4 = t2 * t2;
    T g = t4 * t * (c.C0 + r * (c.C1 + r * (c.C2 + r * c.C3)));
    T h = -t4 * (c.E0 + r * (c.E1 + r * c.E2));
    T j = t3 * (c.F0 * ir + c.F1 + c.F2 * r);
    if (NEAR) {
        // [0, 1] forms
        const T g1 = T(1) + r2 * r * (c.A3 + r2 * (c.A5 + r * (c.A6 + r * (c.A7 + r * c.A8))));
        const T h1 = r * (c.B1 + r2 * (c.B3 + r * (c.B4 + r * (c.B5 + r * c.B6))));
        const T j1 = c.J0 * ir + r * (c.J1 + r * (c.J2 + r * (c.J3 + r * c.J4)));
        const bool inner = r2 < c.rh2;
        g = inner ? g1 : g;
        h = inner ? h1 : h;
        j = inner ? j1 : j;
    }
    const T s3 = u * rinv;
    const T psi = s3 * (h - c.three * u * g);
    const T chi = s3 * (j - u * (c.six * h - c.fifteen * u * g));
    const T sx = s1.x * dx + s1.w * dy + s2.x * dz;
    const T sy = s1.w * dx + s1.y * dy + s2.y * dz;
    const T sz = s2.x * dx + s2.y * dy + s1.z * dz;
    const T dsd = dx * sx + dy * sy + dz * sz;
    const T q = psi * p.w + T(0.5) * chi * dsd;
    ox += psi * sx + q * dx;
    oy += psi * sy + q * dy;
    oz += psi * sz + q * dz;
}

constexpr int kQChunk = 256;   // list entries scanned per compaction round

template <class T>
__global__ __launch_bounds__(64) void k_quadrupole(const int32_t* __restrict__ gfirst,
                                                   const int32_t* __restrict__ gcount,
                                                   const double* __restrict__ glo, const double* __restrict__ ghi,
                                                   const int64_t* __restrict__ off, const int32_t* __restrict__ ent,
                                                   const int32_t* __restrict__ perm, const double* __restrict__ px,
                                                   const double* __restrict__ py, const double* __restrict__ pz,
                                                   const double* __restrict__ nX, const double* __restrict__ nY,
                                                   const double* __restrict__ nZ, const double* __restrict__ S,
                                                   QCoef<T> c, double far2, double G, double* __restrict__ ax,
                                                   double* __restrict__ ay, double* __restrict__ az, int64_t os) {
    using V4 = typename QV4<T>::type;
    using V2 = typename QV2<T>::type;
    __shared__ V4 cp[kQChunk];
    __shared__ V4 cs1[kQChunk];
    __shared__ V2 cs2[kQChunk];
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t first = gfirst[g], cnt = gcount[g];
    const double cx = (glo[g * 3 + 0] + ghi[g * 3 + 0]) * 0.5;
    const double cy = (glo[g * 3 + 1] + ghi[g * 3 + 1]) * 0.5;
    const double cz = (glo[g * 3 + 2] + ghi[g * 3 + 2]) * 0.5;
    const double hx = (ghi[g * 3 + 0] - glo[g * 3 + 0]) * 0.5;
    const double hy = (ghi[g * 3 + 1] - glo[g * 3 + 1]) * 0.5;
    const double hz = (ghi[g * 3 + 2] - glo[g * 3 + 2]) * 0.5;
    const int32_t me = first + (lane < cnt ? lane : 0);
    const T xi = (T)image(px[me] - cx), yi = (T)image(py[me] - cy), zi = (T)image(pz[me] - cz);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const QCoef<T> cq = q_pinned(c);
    double sx = 0, sy = 0, sz = 0;
    const int64_t e0 = off[g], e1 = off[g + 1];
    for (int64_t tb = e0; tb < e1; tb += kQChunk) {
        const int len = (int)((e1 - tb) < kQChunk ? (e1 - tb) : kQChunk);
        __syncthreads();
        // cells compacted: near ones from the front, far ones (distance from
        // the centre of mass to the group box >= r_cut / 2) from the back
        int nnear = 0, nfar = 0;
        for (int k0 = 0; k0 < len; k0 += 64) {
            const int k = k0 + lane;
            const int32_t v = k < len ? ent[tb + k] : 0;
            const bool cell = v < 0;
            double rx = 0, ry = 0, rz = 0;
            bool far = false;
            int64_t q = 0;
            if (cell) {
                q = -(int64_t)v - 1;
                rx = nX[q] - cx;
                ry = nY[q] - cy;
                rz = nZ[q] - cz;
                rx -= rint(rx);
                ry -= rint(ry);
                rz -= rint(rz);
                const double ex = fmax(fabs(rx) - hx, 0.0), ey = fmax(fabs(ry) - hy, 0.0),
                             ez = fmax(fabs(rz) - hz, 0.0);
                far = ex * ex + ey * ey + ez * ez >= far2;
            }
            const uint64_t mn = __ballot(cell && !far), mf = __ballot(cell && far);
            if (cell) {
                const double* s = S + q * 6;
                const int pos = far ? kQChunk - 1 - (nfar + __popcll(mf & lt)) : nnear + __popcll(mn & lt);
                V4 a, b;
                V2 d;
                a.x = (T)rx;
                a.y = (T)ry;
                a.z = (T)rz;
                a.w = (T)(0.5 * (s[0] + s[1] + s[2]));
                b.x = (T)s[0];
                b.y = (T)s[1];
                b.z = (T)s[2];
                b.w = (T)s[3];
                d.x = (T)s[4];
                d.y = (T)s[5];
                cp[pos] = a;
                cs1[pos] = b;
                cs2[pos] = d;
            }
            nnear += __popcll(mn);
            nfar += __popcll(mf);
        }
        __syncthreads();
        T ox = 0, oy = 0, oz = 0;
        for (int k = 0; k < nnear; ++k)
            quad_pair<T, V4, V2, true>(cp[k], cs1[k], cs2[k], xi, yi, zi, cq, ox, oy, oz);
        for (int k = kQChunk - nfar; k < kQChunk; ++k)
            quad_pair<T, V4, V2, false>(cp[k], cs1[k], cs2[k], xi, yi, zi, cq, ox, oy, oz);
        sx += (double)ox;
        sy += (double)oy;
        sz += (double)oz;
    }
    if (lane < cnt) {
        const int64_t o = (int64_t)perm[me] * os;
        ax[o] += G * sx;
        ay[o] += G * sy;
        az[o] += G * sz;
    }
}

}  // namespace

void launch_quadrupole(const Tree& t, const Lists& l, const srf_params& p, double* ax, double* ay, double* az,
                       int64_t os, hipStream_t st) {
    const int64_t nn = t.n_nodes;
    DevBuf<int32_t> used(nn, st);
    DevBuf<double> S(6 * nn, st);
    fill_i32(used.get(), 0, nn, st);
    if (l.n_entries > 0)
        hipLaunchKernelGGL(k_mark_cells, dim3(grid_for(l.n_entries, 256, 1 << 16)), dim3(256), 0, st, l.n_entries,
                           l.ent.get(), used.get());
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_second_moments, dim3((unsigned)((nn + 63) / 64)), dim3(64), 0, st, nn, t.range.get(), used.get(),
                       t.px.get(), t.py.get(), t.pz.get(), t.pm.get(), t.nX.get(), t.nY.get(), t.nZ.get(), S.get());
    SRF_HIP(hipGetLastError());
    const unsigned ng = (unsigned)t.n_groups;
    if (p.precision == SRF_FP64) {
        hipLaunchKernelGGL(k_quadrupole<double>, dim3(ng), dim3(64), 0, st, t.gfirst.get(), t.gcount.get(),
                           t.glo.get(), t.ghi.get(), l.off.get(), l.ent.get(), t.perm.get(), t.px.get(), t.py.get(),
                           t.pz.get(), t.nX.get(), t.nY.get(), t.nZ.get(), S.get(),
                           make_qcoef<double>(p.r_cut, p.eps), 0.25 * p.r_cut * p.r_cut, p.G, ax, ay, az, os);
    } else {
        hipLaunchKernelGGL(k_quadrupole<float>, dim3(ng), dim3(64), 0, st, t.gfirst.get(), t.gcount.get(),
                           t.glo.get(), t.ghi.get(), l.off.get(), l.ent.get(), t.perm.get(), t.px.get(), t.py.get(),
                           t.pz.get(), t.nX.get(), t.nY.get(), t.nZ.get(), S.get(),
                           make_qcoef<float>(p.r_cut, p.eps), 0.25 * p.r_cut * p.r_cut, p.G, ax, ay, az, os);
    }
    SRF_HIP(hipGetLastError());
}

}  // namespace srf
