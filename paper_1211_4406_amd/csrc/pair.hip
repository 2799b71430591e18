// Steps a7-a9: the short-range pair kernel (force and adjoint).
//
// One 64-lane wavefront handles one group.  The group's particles sit in
// registers as offsets from the group centre c_g; the group's list is
// streamed through LDS in tiles of kTile entries, each entry converted once
// (in FP64) to the offset x_j - c_g - rint(x_j - c_g) and stored with its
// mass.  With N_i particles in the group, the wave runs S = floor(64/N_i)
// independent j-streams (lane = i + N_i * stream), whose FP64 partial sums
// are added at the end.  Each staged tile is split into near entries (some
// target may lie within r_cut/2 of them) and far entries (none can); far
// pairs take only the [1,2] form of the cutoff function.
//
// Pair kernel (Sec. 2 force sum with the cutoff function of eq. (cutoff)):
//   phi(r) = (r^2 + eps^2)^(-3/2) g(2 r / r_cut),
//   g(xi) = 1 + xi^3 (-8/5 + xi^2 (8/5 + xi (-1/2 + xi (-12/35 + 3/20 xi))))   xi <= 1
//   g(xi) = t^5 (7 xi^3 + 22 xi^2 + 10 xi + 4) / 140,  t = 2 - xi              1 <= xi <= 2
// (the second line is the printed zeta-branch polynomial in factored form;
// it keeps relative accuracy as g -> 0).  The kernels evaluate both lines
// as one expression (see the arithmetic below) whose factors are clamped so
// that a pair with xi >= 2 in working precision contributes exactly zero:
// no separate cutoff test is needed.  The polynomials are evaluated in r
// with the powers of k = 2/r_cut folded into the coefficients; r is the
// unsoftened distance.
#include <cmath>
#include <mutex>
#include <string>

#include "common.h"

namespace srf {
namespace {

constexpr int kTile = 256;

// ------------------------------------------------------------ arithmetic
// The two pieces of eq. (cutoff) differ on [0,1] by a polynomial that
// vanishes to sixth order at xi = 1:
//   g_[0,1](xi) - g_[1,2](xi) = (1 - xi)^6 (3/35 + 18/35 xi + xi^2/5),
// so with T = 1 - xi/2 and W = 1 - xi, each clamped to [0,1] (T = 0 from
// xi = 2 on, W = 0 from xi = 1 on),
//   g = 32 T^5 R + W^6 Q,  R = (7 xi^3 + 22 xi^2 + 10 xi + 4)/140,
// one expression for every xi with no branch select; both terms are
// nonnegative on [0,2], so the sum loses no accuracy.  The kernels carry
// g/32 (the coefficients absorb the 1/32) and scale by 32 when they convert
// to FP64, which is exact.  A far source (xi >= 1 for every target) takes
// only the T term.
constexpr double kGScale = 32.0;

template <class T>
struct Coef {
    T R0, R1, R2, R3;          // R in r
    T Q0, Q1, Q2;              // Q / 32 in r
    T kh, k;                   // k / 2, k = 2/r_cut
    T eps2;                    // eps^2
    T heps2;                   // -eps^2 / 2
    double far2;               // (r_cut/2)^2 in FP64, for the near/far split of a tile
};

template <class T>
Coef<T> make_coef(double rc, double eps) {
    const double k = 2.0 / rc;
    const double k2 = k * k, k3 = k2 * k;
    Coef<T> c;
    c.R0 = (T)(4.0 / 140.0);
    c.R1 = (T)(10.0 / 140.0 * k);
    c.R2 = (T)(22.0 / 140.0 * k2);
    c.R3 = (T)(7.0 / 140.0 * k3);
    c.Q0 = (T)(3.0 / 35.0 / 32.0);
    c.Q1 = (T)(18.0 / 35.0 / 32.0 * k);
    c.Q2 = (T)(0.2 / 32.0 * k2);
    c.kh = (T)(0.5 * k);
    c.k = (T)k;
    c.eps2 = (T)(eps * eps);
    c.heps2 = (T)(-0.5 * eps * eps);
    c.far2 = 0.25 * rc * rc;
    return c;
}

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float sat_(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }
__device__ __forceinline__ double sat_(double x) { return fmin(fmax(x, 0.0), 1.0); }

// Keep a loop-invariant value in a vector register: the empty asm makes it
// opaque, so the compiler neither folds it back to a scalar operand nor
// re-materialises it inside the pair loops (a VALU op may read at most one
// scalar operand, so scalar constants would otherwise cost moves per pair).
__device__ __forceinline__ float pin_(float x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ double pin_(double x) {
    asm volatile("" : "+v"(x));
    return x;
}

template <class T>
__device__ __forceinline__ Coef<T> pinned(const Coef<T>& a) {
    Coef<T> c;
    c.R0 = pin_(a.R0); c.R1 = pin_(a.R1); c.R2 = pin_(a.R2); c.R3 = pin_(a.R3);
    c.Q0 = pin_(a.Q0); c.Q1 = pin_(a.Q1); c.Q2 = pin_(a.Q2);
    c.kh = pin_(a.kh); c.k = pin_(a.k); c.eps2 = pin_(a.eps2); c.heps2 = pin_(a.heps2);
    c.far2 = a.far2;
    return c;
}

template <class T>
struct Vec4 {};
template <>
struct Vec4<float> { using type = float4; };
template <>
struct Vec4<double> { using type = double4; };

// g/32 for one pair, from r (0 at and beyond xi = 2 through the clamp of T).
template <class T>
__device__ __forceinline__ T cutoff_g(T r, const Coef<T>& c) {
    const T t = sat_(fma_(r, -c.kh, T(1)));
    const T w = sat_(fma_(r, -c.k, T(1)));
    const T R = fma_(fma_(fma_(r, c.R3, c.R2), r, c.R1), r, c.R0);
    const T Q = fma_(fma_(r, c.Q2, c.Q1), r, c.Q0);
    const T t2 = t * t, w2 = w * w;
    return fma_((w2 * w2) * w2, Q, (t2 * t2) * (t * R));
}

// FP32 partial sums of one target over a tile.  With COMP each component
// carries a Kahan compensation term (sum = a - c).
template <class T, bool COMP>
struct Acc {
    T x = 0, y = 0, z = 0;
    T cx = 0, cy = 0, cz = 0;
    __device__ __forceinline__ static void add1(T& a, T& c, T v) {
        if (COMP) {
            const T y = v - c;
            const T t = a + y;
            c = (t - a) - y;
            a = t;
        } else {
            a += v;
        }
    }
    // the partials, times 32 (g/32 was summed), added to FP64 totals
    __device__ __forceinline__ void flush(double& sx, double& sy, double& sz) const {
        sx += kGScale * (COMP ? (double)x - (double)cx : (double)x);
        sy += kGScale * (COMP ? (double)y - (double)cy : (double)y);
        sz += kGScale * (COMP ? (double)z - (double)cz : (double)z);
    }
    __device__ __forceinline__ void add(T f, T dx, T dy, T dz) {
        if (COMP) {
            add1(x, cx, f * dx);
            add1(y, cy, f * dy);
            add1(z, cz, f * dz);
        } else {
            x = fma_(f, dx, x);
            y = fma_(f, dy, y);
            z = fma_(f, dz, z);
        }
    }
};

// Unsoftened distance r of a far pair from s^2 = r^2 + eps^2 and s^-1.  With
// RS it is r = s - eps^2 / (2 s) = s^2 s^-1 - (eps^2 / 2) s^-1, whose
// relative error is y^2/8 + O(y^3) with y = eps^2 / s^2 <= (2 eps / r_cut)^2
// for far pairs (s >= r_cut / 2); the host selects RS only when that bound
// keeps the error below half an FP32 ulp.  Otherwise r = sqrt(r^2).
template <class T, bool RS, class C>
__device__ __forceinline__ T far_r(T r2, T s2, T rinv, const C& c) {
    return RS ? fma_(c.heps2, rinv, s2 * rinv) : sqrt_(r2);
}

// Force of one source (offset p.xyz, mass p.w) on one target (xi, yi, zi),
// divided by 32, accumulated into acc.  NEAR selects the full cutoff
// function; otherwise the source lies at xi >= 1 from the target,
// g/32 = T^5 R, and the factor m s^-3 T^5 R is formed as m (q^2)(q T)(T R)
// with q = T s^-1.
template <class T, class V4, bool NEAR, bool COMP, bool RS>
__device__ __forceinline__ void pair_force(const V4& p, T xi, T yi, T zi, const Coef<T>& c, Acc<T, COMP>& acc) {
    const T dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
    // the far path with r from s needs no unsoftened r^2: s^2 directly
    const bool direct = !NEAR && RS;
    const T r2 = direct ? T(0) : fma_(dz, dz, fma_(dy, dy, dx * dx));
    const T s2 = direct ? fma_(dz, dz, fma_(dy, dy, fma_(dx, dx, c.eps2))) : r2 + c.eps2;
    const T rinv = rsqrt_(s2);
    const T r = NEAR ? sqrt_(r2) : far_r<T, RS>(r2, s2, rinv, c);
    T f;
    if (NEAR) {
        const T g = cutoff_g(r, c);
        f = (p.w * rinv) * (rinv * rinv) * g;
    } else {
        const T t = sat_(fma_(r, -c.kh, T(1)));
        const T R = fma_(fma_(fma_(r, c.R3, c.R2), r, c.R1), r, c.R0);
        const T q = t * rinv;
        f = p.w * ((q * q) * ((q * t) * (t * R)));
    }
    acc.add(f, dx, dy, dz);
}

// ------------------------------------------------------------ tile loading
struct Src {
    const double *px, *py, *pz, *pm;
    const double *nX, *nY, *nZ, *nM;
};

// Load one list entry (particle v >= 0, or cell -v-1 as its monopole) as
// the FP32 offset x_j - c - rint(x_j - c) from the group centre c, with its
// mass, and classify it: far when its distance to the group's box (half
// extents h) is at least r_cut/2, so that xi >= 1 holds for every target of
// the group.  The distance is the FP64 distance from the source point
// (particle or centre of mass) to the box.
template <class T, class V4>
__device__ __forceinline__ V4 load_entry_cls(int32_t v, const Src& s, double cx, double cy, double cz, double hx,
                                             double hy, double hz, double far2, bool& far) {
    double X, Y, Z, M;
    if (v >= 0) {
        X = s.px[v];
        Y = s.py[v];
        Z = s.pz[v];
        M = s.pm[v];
    } else {
        const int32_t c = -v - 1;
        X = s.nX[c];
        Y = s.nY[c];
        Z = s.nZ[c];
        M = s.nM[c];
    }
    double rx = X - cx, ry = Y - cy, rz = Z - cz;
    rx -= rint(rx);
    ry -= rint(ry);
    rz -= rint(rz);
    const double ex = fmax(fabs(rx) - hx, 0.0), ey = fmax(fabs(ry) - hy, 0.0), ez = fmax(fabs(rz) - hz, 0.0);
    far = ex * ex + ey * ey + ez * ez >= far2;
    V4 o;
    o.x = (T)rx;
    o.y = (T)ry;
    o.z = (T)rz;
    o.w = (T)M;
    return o;
}

// Stage one tile of a group's list in LDS, near entries first (slots
// [0, n_near)) and far entries after them (filled from the end).  Returns
// n_near; the order within each class is fixed by the list, so the result
// is deterministic.  An entry that is one of the group's own particles is
// near.  `ids`, if given, receives each entry's row in the adjoint's
// source array (particle s -> s, cell c -> n_part + c).  The PAD slots after
// the last entry are set to zero mass at the origin (row -1), so that a
// read past the end of a segment stays finite.
template <class T, class V4, int PAD = 0>
__device__ __forceinline__ int stage_tile(const int32_t* __restrict__ ent, int len, const Src& src, double cx,
                                          double cy, double cz, double hx, double hy, double hz, double far2,
                                          V4* tile, int32_t* ids, int32_t n_part = 0) {
    const int lane = threadIdx.x;
    if (PAD > 0 && lane < PAD) {
        V4 z;
        z.x = z.y = z.z = z.w = T(0);
        tile[len + lane] = z;
        if (ids) ids[len + lane] = -1;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int nnear = 0, nfar = 0;
    for (int k0 = 0; k0 < len; k0 += 64) {
        const int k = k0 + lane;
        const bool valid = k < len;
        bool far = false;
        V4 e;
        int32_t v = 0;
        if (valid) {
            v = ent[k];
            e = load_entry_cls<T, V4>(v, src, cx, cy, cz, hx, hy, hz, far2, far);
        }
        const uint64_t mn = __ballot(valid && !far), mf = __ballot(valid && far);
        if (valid) {
            const int pos = far ? len - 1 - (nfar + __popcll(mf & lt)) : nnear + __popcll(mn & lt);
            tile[pos] = e;
            if (ids) ids[pos] = v >= 0 ? v : n_part + (-v - 1);
        }
        nnear += __popcll(mn);
        nfar += __popcll(mf);
    }
    return nnear;
}

// Pairs of this lane's stream with the entries [a, b) of a staged tile
// (entries a + st, a + st + S, ...).  The unrolled loop takes U entries
// per stream (8 for the shorter far pairs, 4 for near pairs) while all
// streams have U left, so its trip count is the same for every lane.  The
// FP32 partial sums are added to the FP64 totals every kFlush entries:
// the rounding error of an FP32 running sum grows with its length, and on
// near-uniform sets, where a particle's force is a small residual of its
// neighbours' pulls, partials over a whole tile (256 entries) dominated the
// error; chunks of 32 cost no measurable time.
constexpr int kFlush = 32;
template <class T, class V4, int S, bool NEAR, bool COMP, bool RS>
__device__ __forceinline__ void force_segment(const V4* tile, int a, int b, int st, T xi, T yi, T zi,
                                              const Coef<T>& c, double& sx, double& sy, double& sz) {
    constexpr int U = NEAR ? 4 : 8;
    constexpr int FL = kFlush / U;
    const V4* tp = tile + a + st;
    int kk = a;
    while (kk + U * S <= b) {
        Acc<T, COMP> acc;
        for (int it = 0; it < FL && kk + U * S <= b; ++it, kk += U * S, tp += U * S) {
            V4 pp[U];
#pragma unroll
            for (int u = 0; u < U; ++u) pp[u] = tp[u * S];
#pragma unroll
            for (int u = 0; u < U; ++u) pair_force<T, V4, NEAR, COMP, RS>(pp[u], xi, yi, zi, c, acc);
        }
        acc.flush(sx, sy, sz);
    }
    Acc<T, COMP> acc;
    for (int k = kk + st; k < b; k += S, tp += S) pair_force<T, V4, NEAR, COMP, RS>(tp[0], xi, yi, zi, c, acc);
    acc.flush(sx, sy, sz);
}

struct GroupArgs {
    const int32_t *gfirst, *gcount;
    const double *glo, *ghi;
    const int64_t* off;
    const int32_t* ent;
    const int32_t* perm;
};

// ------------------------------------------------------------------ force
template <class T, int S, bool COMP, bool RS>
__device__ __forceinline__ void force_group(const GroupArgs& ga, const Src& src, const Coef<T>& c0, double G,
                                            double* __restrict__ ax, double* __restrict__ ay,
                                            double* __restrict__ az, int64_t os, int64_t g, int32_t first,
                                            int32_t cnt, typename Vec4<T>::type* tile, double* red) {
    using V4 = typename Vec4<T>::type;
    const Coef<T> c = pinned(c0);
    const int lane = threadIdx.x;
    const int il = lane % cnt, st = lane / cnt;
    const bool active = st < S;
    const double cx = (ga.glo[g * 3 + 0] + ga.ghi[g * 3 + 0]) * 0.5;
    const double cy = (ga.glo[g * 3 + 1] + ga.ghi[g * 3 + 1]) * 0.5;
    const double cz = (ga.glo[g * 3 + 2] + ga.ghi[g * 3 + 2]) * 0.5;
    const double hx = (ga.ghi[g * 3 + 0] - ga.glo[g * 3 + 0]) * 0.5;
    const double hy = (ga.ghi[g * 3 + 1] - ga.glo[g * 3 + 1]) * 0.5;
    const double hz = (ga.ghi[g * 3 + 2] - ga.glo[g * 3 + 2]) * 0.5;
    const int32_t me = first + il;
    const T xi = (T)image(src.px[me] - cx), yi = (T)image(src.py[me] - cy), zi = (T)image(src.pz[me] - cz);
    double sx = 0, sy = 0, sz = 0;
    const int64_t e0 = ga.off[g], e1 = ga.off[g + 1];
    for (int64_t tb = e0; tb < e1; tb += kTile) {
        const int len = (int)((e1 - tb) < kTile ? (e1 - tb) : kTile);
        __syncthreads();
        const int nnear = stage_tile<T, V4>(ga.ent + tb, len, src, cx, cy, cz, hx, hy, hz, c0.far2, tile, nullptr);
        __syncthreads();
        if (active) {
            force_segment<T, V4, S, true, COMP, RS>(tile, 0, nnear, st, xi, yi, zi, c, sx, sy, sz);
            force_segment<T, V4, S, false, COMP, RS>(tile, nnear, len, st, xi, yi, zi, c, sx, sy, sz);
        }
    }
    red[lane * 3 + 0] = sx;
    red[lane * 3 + 1] = sy;
    red[lane * 3 + 2] = sz;
    __syncthreads();
    if (lane < cnt) {
        double tx = 0, ty = 0, tz = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int l = lane + q * cnt;
            tx += red[l * 3 + 0];
            ty += red[l * 3 + 1];
            tz += red[l * 3 + 2];
        }
        const int64_t o = (int64_t)ga.perm[me] * os;
        ax[o] = G * tx;
        ay[o] = G * ty;
        az[o] = G * tz;
    }
}

// Streams per group: the largest of 1, 2, 3, 4, 8 with S * N_i <= 64.
template <class T, bool COMP, bool RS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_force(
    GroupArgs ga, Src src, Coef<T> c, double G, double* __restrict__ ax, double* __restrict__ ay,
    double* __restrict__ az, int64_t os) {
    using V4 = typename Vec4<T>::type;
    __shared__ V4 tile[kTile];
    __shared__ double red[64 * 3];
    const int64_t g = xcd_block(blockIdx.x, gridDim.x);
    const int32_t first = ga.gfirst[g], cnt = ga.gcount[g];
    if (cnt > 32) force_group<T, 1, COMP, RS>(ga, src, c, G, ax, ay, az, os, g, first, cnt, tile, red);
    else if (cnt > 21) force_group<T, 2, COMP, RS>(ga, src, c, G, ax, ay, az, os, g, first, cnt, tile, red);
    else if (cnt > 16) force_group<T, 3, COMP, RS>(ga, src, c, G, ax, ay, az, os, g, first, cnt, tile, red);
    else if (cnt > 8) force_group<T, 4, COMP, RS>(ga, src, c, G, ax, ay, az, os, g, first, cnt, tile, red);
    else force_group<T, 8, COMP, RS>(ga, src, c, G, ax, ay, az, os, g, first, cnt, tile, red);
}

// -------------------------------------------------------------- potential
// Short-range potential of the split, -G sum_j m_j q(xi) / s (the target
// left out), with q the potential factor of the pair force (g = q - xi q'):
//   q(xi) = 1 - 52/35 xi + 4/5 xi^3 - 2/5 xi^5 + 1/10 xi^6 + 2/35 xi^7 - 3/140 xi^8   xi <= 1
//   q(xi) = (2 - xi)^6 (xi^2 + 4 xi + 2) / 140                                       1 <= xi <= 2
// evaluated in r with the powers of k folded into the coefficients, as g.
template <class T>
struct PotCoef {
    T D1, D3, D5, D6, D7, D8;   // q on [0,1] - 1, in r
    T Q0, Q1, Q2;               // (xi^2 + 4 xi + 2) / 140 in r
    T k, eps2, rh2, heps2;
    double far2;
};

template <class T>
PotCoef<T> make_pot_coef(double rc, double eps) {
    const double k = 2.0 / rc;
    PotCoef<T> c;
    c.D1 = (T)(-52.0 / 35.0 * k);
    c.D3 = (T)(0.8 * k * k * k);
    c.D5 = (T)(-0.4 * pow(k, 5));
    c.D6 = (T)(0.1 * pow(k, 6));
    c.D7 = (T)(2.0 / 35.0 * pow(k, 7));
    c.D8 = (T)(-3.0 / 140.0 * pow(k, 8));
    c.Q0 = (T)(2.0 / 140.0);
    c.Q1 = (T)(4.0 / 140.0 * k);
    c.Q2 = (T)(1.0 / 140.0 * k * k);
    c.k = (T)k;
    c.eps2 = (T)(eps * eps);
    c.rh2 = (T)(0.25 * rc * rc);
    c.heps2 = (T)(-0.5 * eps * eps);
    c.far2 = 0.25 * rc * rc;
    return c;
}

template <class T>
__device__ __forceinline__ PotCoef<T> pinned(const PotCoef<T>& a) {
    PotCoef<T> c;
    c.D1 = pin_(a.D1); c.D3 = pin_(a.D3); c.D5 = pin_(a.D5); c.D6 = pin_(a.D6); c.D7 = pin_(a.D7);
    c.D8 = pin_(a.D8); c.Q0 = pin_(a.Q0); c.Q1 = pin_(a.Q1); c.Q2 = pin_(a.Q2);
    c.k = pin_(a.k); c.eps2 = pin_(a.eps2); c.rh2 = pin_(a.rh2); c.heps2 = pin_(a.heps2);
    c.far2 = a.far2;
    return c;
}

// m q(xi) / s for one source (offset p.xyz, mass p.w); `self` leaves the
// target's own entry out.
template <class T, class V4, bool NEAR, bool RS>
__device__ __forceinline__ T pair_pot(const V4& p, T xi, T yi, T zi, const PotCoef<T>& c, bool self) {
    const T dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
    const T r2 = fma_(dz, dz, fma_(dy, dy, dx * dx));
    const T s2 = r2 + c.eps2;
    const T rinv = (NEAR && self) ? T(0) : rsqrt_(s2);
    T r;
    if (NEAR) r = sqrt_(r2);
    else r = RS ? fma_(c.heps2, rinv, s2 * rinv) : sqrt_(r2);
    const T t = sat_(fma_(r, -c.k, T(2)));
    const T t2 = t * t;
    const T q2 = (t2 * t2) * t2 * fma_(fma_(r, c.Q2, c.Q1), r, c.Q0);
    T q = q2;
    if (NEAR) {
        T u = fma_(r, c.D8, c.D7);
        u = fma_(r, u, c.D6);
        u = fma_(r, u, c.D5);
        u = fma_(r2, u, c.D3);
        u = fma_(r2, u, c.D1);
        const T q1 = fma_(r, u, T(1));
        q = r2 < c.rh2 ? q1 : q2;
    }
    return p.w * q * rinv;
}

template <class T, int S, bool RS>
__device__ __forceinline__ void potential_group(const GroupArgs& ga, const Src& src, const PotCoef<T>& c0, double G,
                                                double* __restrict__ phi, int64_t os, int32_t n_part, int64_t g,
                                                int32_t first, int32_t cnt, typename Vec4<T>::type* tile,
                                                int32_t* ids, double* red) {
    using V4 = typename Vec4<T>::type;
    const PotCoef<T> c = pinned(c0);
    const int lane = threadIdx.x;
    const int il = lane % cnt, st = lane / cnt;
    const bool active = st < S;
    const double cx = (ga.glo[g * 3 + 0] + ga.ghi[g * 3 + 0]) * 0.5;
    const double cy = (ga.glo[g * 3 + 1] + ga.ghi[g * 3 + 1]) * 0.5;
    const double cz = (ga.glo[g * 3 + 2] + ga.ghi[g * 3 + 2]) * 0.5;
    const double hx = (ga.ghi[g * 3 + 0] - ga.glo[g * 3 + 0]) * 0.5;
    const double hy = (ga.ghi[g * 3 + 1] - ga.glo[g * 3 + 1]) * 0.5;
    const double hz = (ga.ghi[g * 3 + 2] - ga.glo[g * 3 + 2]) * 0.5;
    const int32_t me = first + il;
    const T xi = (T)image(src.px[me] - cx), yi = (T)image(src.py[me] - cy), zi = (T)image(src.pz[me] - cz);
    double sum = 0.0;
    const int64_t e0 = ga.off[g], e1 = ga.off[g + 1];
    for (int64_t tb = e0; tb < e1; tb += kTile) {
        const int len = (int)((e1 - tb) < kTile ? (e1 - tb) : kTile);
        __syncthreads();
        const int nnear = stage_tile<T, V4>(ga.ent + tb, len, src, cx, cy, cz, hx, hy, hz, c0.far2, tile, ids,
                                            n_part);
        __syncthreads();
        if (active) {
            // FP32 partials over at most kFlush entries of this lane, added in FP64
            for (int k0 = st; k0 < nnear; k0 += kFlush * S) {
                const int k1 = k0 + kFlush * S < nnear ? k0 + kFlush * S : nnear;
                T acc = 0;
                for (int k = k0; k < k1; k += S) acc += pair_pot<T, V4, true, RS>(tile[k], xi, yi, zi, c, ids[k] == me);
                sum += (double)acc;
            }
            for (int k0 = nnear + st; k0 < len; k0 += kFlush * S) {
                const int k1 = k0 + kFlush * S < len ? k0 + kFlush * S : len;
                T acc = 0;
                for (int k = k0; k < k1; k += S) acc += pair_pot<T, V4, false, RS>(tile[k], xi, yi, zi, c, false);
                sum += (double)acc;
            }
        }
    }
    red[lane] = active ? sum : 0.0;
    __syncthreads();
    if (lane < cnt) {
        double tot = 0.0;
#pragma unroll
        for (int q = 0; q < S; ++q) tot += red[lane + q * cnt];
        phi[(int64_t)ga.perm[me] * os] = -G * tot;
    }
}

// Streams per group as in the force kernel.  `n_part` is the particle count
// (the staged rows of cells start there, so that no cell matches a target).
template <class T, bool RS>
__global__ __launch_bounds__(64) void k_potential(GroupArgs ga, Src src, PotCoef<T> c, double G,
                                                  double* __restrict__ phi, int64_t os, int32_t n_part) {
    using V4 = typename Vec4<T>::type;
    __shared__ V4 tile[kTile];
    __shared__ int32_t ids[kTile];
    __shared__ double red[64];
    const int64_t g = xcd_block(blockIdx.x, gridDim.x);
    const int32_t first = ga.gfirst[g], cnt = ga.gcount[g];
    if (cnt > 32) potential_group<T, 1, RS>(ga, src, c, G, phi, os, n_part, g, first, cnt, tile, ids, red);
    else if (cnt > 21) potential_group<T, 2, RS>(ga, src, c, G, phi, os, n_part, g, first, cnt, tile, ids, red);
    else if (cnt > 16) potential_group<T, 3, RS>(ga, src, c, G, phi, os, n_part, g, first, cnt, tile, ids, red);
    else if (cnt > 8) potential_group<T, 4, RS>(ga, src, c, G, phi, os, n_part, g, first, cnt, tile, ids, red);
    else potential_group<T, 8, RS>(ga, src, c, G, phi, os, n_part, g, first, cnt, tile, ids, red);
}

// ---------------------------------------------------------------- adjoint
// For a pair (target i with weight w, source of mass mu at offset d):
//   V = J(d) w = phi w + psi (d . w) d,  psi = phi'(r) / r,
//   dL/dx_i -= mu V,   dL/dy_src += mu V,   dL/dmu_src += phi (d . w).
// A self pair (the target itself in its list; the force sum is over j != i)
// gets s^-1 = 0, so phi and psi vanish.
// phi = s^-3 g and psi = phi'(r) / r = s^-3 (h - 3 s^-2 g), h = k^2 g'(xi)/xi.
// With g in the one-expression form of the force kernel (T and W as there),
// the derivatives of the two pieces of eq. (cutoff) differ on [0,1] by
//   (g'_[0,1] - g'_[1,2]) / xi = (1 - xi)^5 (-16/5 - 8/5 xi),
// so h = -16 T^4 P + W^5 L with P = k^2 (2 xi^2 + 4 xi - 1)/5 and L = k^2
// times the polynomial above.  The kernel carries phi/32 and psi/32 and
// scales by 32 in FP64.  A far source takes only the T terms.
template <class T>
struct AdjCoef {
    T R0, R1, R2, R3;          // R in r
    T P0, P1, P2;              // P / 2 in r
    T Q0, Q1, Q2;              // Q / 32 in r
    T L0, L1;                  // k^2 L / 32 in r
    T kh, k;                   // k / 2, k = 2 / r_cut
    T eps2, heps2, m3;         // eps^2, -eps^2 / 2, -3
    double far2;               // (r_cut/2)^2 in FP64, for the near/far split of a tile
};

template <class T>
AdjCoef<T> make_adj_coef(double rc, double eps) {
    const double k = 2.0 / rc;
    const double k2 = k * k, k3 = k2 * k, k4 = k3 * k;
    AdjCoef<T> c;
    c.R0 = (T)(4.0 / 140.0);
    c.R1 = (T)(10.0 / 140.0 * k);
    c.R2 = (T)(22.0 / 140.0 * k2);
    c.R3 = (T)(7.0 / 140.0 * k3);
    c.P0 = (T)(-0.1 * k2);
    c.P1 = (T)(0.4 * k3);
    c.P2 = (T)(0.2 * k4);
    c.Q0 = (T)(3.0 / 35.0 / 32.0);
    c.Q1 = (T)(18.0 / 35.0 / 32.0 * k);
    c.Q2 = (T)(0.2 / 32.0 * k2);
    c.L0 = (T)(-3.2 / 32.0 * k2);
    c.L1 = (T)(-1.6 / 32.0 * k3);
    c.kh = (T)(0.5 * k);
    c.k = (T)k;
    c.eps2 = (T)(eps * eps);
    c.heps2 = (T)(-0.5 * eps * eps);
    c.m3 = (T)(-3.0);
    c.far2 = 0.25 * rc * rc;
    return c;
}

template <class T>
__device__ __forceinline__ AdjCoef<T> pinned(const AdjCoef<T>& a) {
    AdjCoef<T> c;
    c.R0 = pin_(a.R0); c.R1 = pin_(a.R1); c.R2 = pin_(a.R2); c.R3 = pin_(a.R3);
    c.P0 = pin_(a.P0); c.P1 = pin_(a.P1); c.P2 = pin_(a.P2);
    c.Q0 = pin_(a.Q0); c.Q1 = pin_(a.Q1); c.Q2 = pin_(a.Q2);
    c.L0 = pin_(a.L0); c.L1 = pin_(a.L1);
    c.kh = pin_(a.kh); c.k = pin_(a.k);
    c.eps2 = pin_(a.eps2); c.heps2 = pin_(a.heps2); c.m3 = pin_(a.m3);
    c.far2 = a.far2;
    return c;
}

// phi/32 and psi/32 of one pair from r and s^-1.
template <class T, bool NEAR>
__device__ __forceinline__ void jac_coefs(T r, T rinv, const AdjCoef<T>& c, T& phi, T& psi) {
    const T u = rinv * rinv;
    const T s3 = u * rinv;
    const T t = sat_(fma_(r, -c.kh, T(1)));
    const T R = fma_(fma_(fma_(r, c.R3, c.R2), r, c.R1), r, c.R0);
    const T P = fma_(fma_(r, c.P2, c.P1), r, c.P0);
    const T t4 = (t * t) * (t * t);
    if (NEAR) {
        const T w = sat_(fma_(r, -c.k, T(1)));
        const T w2 = w * w;
        const T w4 = w2 * w2;
        const T Q = fma_(fma_(r, c.Q2, c.Q1), r, c.Q0);
        const T L = fma_(r, c.L1, c.L0);
        const T g = fma_(w4 * w2, Q, t4 * (t * R));
        const T h = fma_(w4 * w, L, -(t4 * P));
        phi = s3 * g;
        psi = s3 * fma_(c.m3 * u, g, h);
    } else {
        // g = T^4 (T R), h = -T^4 P; with a = s^-3 T^4:
        // phi = a (T R), psi = -3 u phi - a P
        const T a = s3 * t4;
        phi = a * (t * R);
        psi = fma_(c.m3 * u, phi, -(a * P));
    }
}

struct AdjOut {
    double *gix, *giy, *giz;            // i-side, sorted order (plain stores)
    double *gj;                         // j-side, [n + n_nodes][4] = (x, y, z, m), atomics:
                                        // row s for particle s, row n + c for cell c
    double *gn;                         // = gj + 4 n, the cell rows
    int64_t n, nn;
};

// Adjoint pair pass.  The wave is laid out as 4 rows of 16 lanes: lane
// (a, b) = (lane & 15, lane >> 4).  Targets are taken in NB blocks of 16
// (target 16 ib + a in block ib, NB = ceil(N_i / 16)), entries in blocks of
// 4 (entry b of the block on row b).  For one entry block a lane evaluates
// its entry against its target of each of the NB target blocks:
//   - the i-side term -mu V goes to the lane's FP32 accumulator of that
//     target (summed over the rows once per tile, in FP64, into the FP64
//     total the target's own lane keeps),
//   - V = J w_i and phi (d . w_i) are summed in registers over the NB
//     blocks; the lane stores these four partial sums in LDS, and after
//     every four entry blocks each lane adds the 16 partials of one (entry,
//     value), scales the entry's V by its mass and adds the total to the
//     source's gradient with an FP64 atomic (the stores and reads are LDS
//     operations, which issue beside the vector ALU; a sum across the row's
//     lanes in registers costs 6 selects and 5 DPP adds per block).
// Targets past N_i carry zero weight, so they add nothing to either side.
constexpr int kRow = 16;   // lanes per row: targets per block
constexpr int kRows = 4;   // rows: entries per block

// Targets of one lane: block ib holds target 16 ib + a.
template <class T, int NB>
struct Targets {
    T x[NB], y[NB], z[NB], wx[NB], wy[NB], wz[NB];
    // i-side partial sums over the tile: A = sum mu phi, B = sum mu psi (d . w) d,
    // so that -sum mu V = -(A w + B)
    T A[NB], Bx[NB], By[NB], Bz[NB];
    int32_t id[NB];     // sorted particle index, for the self test
};

// Entry blocks [a, b) of a staged tile (all near or all far).  Slots past
// b hold entries of the next segment or the zero padding: their mass is
// taken as zero, and their j-side sums are not added (the segment that owns
// them adds its own).
// Row sums through LDS: after each entry block a lane stores its four
// partial sums in `part` ([block][value][row][16], each [row][16] group
// followed by one padding word, so that both the stores of one value by the
// 64 lanes and the reads of one partial index by them fall on distinct
// banks in pairs); after every kGroupBlocks blocks (and at the segment's end)
// lane (block, value, row) adds the row's 16 partials, and the totals of
// (mu V_x, mu V_y, mu V_z, sum phi (d . w)) of each entry go to row ids[e]
// of the j-side array with FP64 atomics (a zero, every pair of the entry
// beyond r_cut, is not added).
constexpr int kGroupBlocks = 4;
constexpr int kPartRow = kRow;                     // one row's 16 partials
constexpr int kPartValue = kRows * kPartRow + 1;   // one value of a block: 4 rows + padding
constexpr int kPartBlock = 4 * kPartValue;

__device__ __forceinline__ void lds_order() {
    // one wave: its LDS operations complete in order; this keeps the
    // compiler from moving them across
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T, class V4, int NB, bool NEAR, bool RS>
__device__ __forceinline__ void adjoint_entries(int a, int b, const V4* tile, const int32_t* ids,
                                                double* __restrict__ gj, T* part, int lane, Targets<T, NB>& tg,
                                                const AdjCoef<T>& c) {
    const int ra = lane & (kRow - 1), rb = lane >> 4;
    int nblk = 0, eb0 = a;
    T* wp = part + rb * kPartRow + ra;
    // this lane's sum in the reduction: block, value, row
    const int sb = lane >> 4, sv = (lane >> 2) & 3, sr = lane & 3;
    const T* rp = part + sb * kPartBlock + sv * kPartValue + sr * kPartRow;
    for (int eb = a; eb < b; eb += kRows) {
        const int e = eb + rb;
        V4 p = tile[e];
        p.w = e < b ? p.w : T(0);
        const int32_t v = NEAR ? ids[e] : 0;
        T jx, jy, jz, jm;
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
            const T dx = p.x - tg.x[ib], dy = p.y - tg.y[ib], dz = p.z - tg.z[ib];
            // the far path with r from s needs no unsoftened r^2: s^2 directly
            const bool direct = !NEAR && RS;
            const T r2 = direct ? T(0) : fma_(dz, dz, fma_(dy, dy, dx * dx));
            const T s2 = direct ? fma_(dz, dz, fma_(dy, dy, fma_(dx, dx, c.eps2))) : r2 + c.eps2;
            const T rinv = (NEAR && v == tg.id[ib]) ? T(0) : rsqrt_(s2);
            const T r = NEAR ? sqrt_(r2) : far_r<T, RS>(r2, s2, rinv, c);
            T phi, psi;
            jac_coefs<T, NEAR>(r, rinv, c, phi, psi);
            const T dw = fma_(dz, tg.wz[ib], fma_(dy, tg.wy[ib], dx * tg.wx[ib]));
            const T s = psi * dw;
            const T ms = p.w * s;
            tg.A[ib] = fma_(p.w, phi, tg.A[ib]);
            tg.Bx[ib] = fma_(ms, dx, tg.Bx[ib]);
            tg.By[ib] = fma_(ms, dy, tg.By[ib]);
            tg.Bz[ib] = fma_(ms, dz, tg.Bz[ib]);
            // j-side: V = phi w + s d and phi (d . w), summed over the targets
            if (ib == 0) {
                jx = fma_(s, dx, phi * tg.wx[ib]);
                jy = fma_(s, dy, phi * tg.wy[ib]);
                jz = fma_(s, dz, phi * tg.wz[ib]);
                jm = phi * dw;
            } else {
                jx = fma_(s, dx, fma_(phi, tg.wx[ib], jx));
                jy = fma_(s, dy, fma_(phi, tg.wy[ib], jy));
                jz = fma_(s, dz, fma_(phi, tg.wz[ib], jz));
                jm = fma_(phi, dw, jm);
            }
        }
        T* w = wp + nblk * kPartBlock;
        w[0] = jx;
        w[kPartValue] = jy;
        w[2 * kPartValue] = jz;
        w[3 * kPartValue] = jm;
        ++nblk;
        if (nblk == kGroupBlocks || eb + kRows >= b) {
            lds_order();
            const int e = eb0 + kRows * sb + sr;
            if (sb < nblk && e < b) {
                T sum = rp[0];
#pragma unroll
                for (int q = 1; q < kRow; ++q) sum += rp[q];
                const T val = sv == 3 ? sum : sum * tile[e].w;
                if (val != T(0)) unsafeAtomicAdd(gj + (4 * (int64_t)ids[e] + sv), kGScale * (double)val);
            }
            lds_order();
            nblk = 0;
            eb0 = eb + kRows;
        }
    }
}

template <class T, int NB, bool RS>
__device__ __forceinline__ void adjoint_group(const GroupArgs& ga, const Src& src, const AdjCoef<T>& c0,
                                              const double* __restrict__ wx, const double* __restrict__ wy,
                                              const double* __restrict__ wz, int64_t ws, const AdjOut& out,
                                              int64_t g, int32_t first, int32_t cnt,
                                              typename Vec4<T>::type* tile, int32_t* ids, T* part) {
    using V4 = typename Vec4<T>::type;
    const AdjCoef<T> c = pinned(c0);
    const int lane = threadIdx.x;
    const int ra = lane & (kRow - 1), rb = lane >> 4;
    const double cx = (ga.glo[g * 3 + 0] + ga.ghi[g * 3 + 0]) * 0.5;
    const double cy = (ga.glo[g * 3 + 1] + ga.ghi[g * 3 + 1]) * 0.5;
    const double cz = (ga.glo[g * 3 + 2] + ga.ghi[g * 3 + 2]) * 0.5;
    const double hx = (ga.ghi[g * 3 + 0] - ga.glo[g * 3 + 0]) * 0.5;
    const double hy = (ga.ghi[g * 3 + 1] - ga.glo[g * 3 + 1]) * 0.5;
    const double hz = (ga.ghi[g * 3 + 2] - ga.glo[g * 3 + 2]) * 0.5;
    Targets<T, NB> tg;
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
        const int i = ib * kRow + ra;
        const int32_t me = first + (i < cnt ? i : 0);
        tg.x[ib] = (T)image(src.px[me] - cx);
        tg.y[ib] = (T)image(src.py[me] - cy);
        tg.z[ib] = (T)image(src.pz[me] - cz);
        const int64_t wi = (int64_t)ga.perm[me] * ws;
        const bool on = i < cnt;
        tg.wx[ib] = on ? (T)wx[wi] : T(0);
        tg.wy[ib] = on ? (T)wy[wi] : T(0);
        tg.wz[ib] = on ? (T)wz[wi] : T(0);
        tg.id[ib] = on ? first + i : INT32_MIN;   // INT32_MIN is no list value
    }
    // FP64 i-side total of target `lane` (block rb, slot ra), kept by that lane
    double gx = 0.0, gy = 0.0, gz = 0.0;
    const int64_t e0 = ga.off[g], e1 = ga.off[g + 1];
    for (int64_t tb = e0; tb < e1; tb += kTile) {
        const int len = (int)((e1 - tb) < kTile ? (e1 - tb) : kTile);
        __syncthreads();
        const int nnear = stage_tile<T, V4, kRows>(ga.ent + tb, len, src, cx, cy, cz, hx, hy, hz, c0.far2, tile, ids,
                                                   (int32_t)out.n);
        __syncthreads();
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) tg.A[ib] = tg.Bx[ib] = tg.By[ib] = tg.Bz[ib] = T(0);
        adjoint_entries<T, V4, NB, true, RS>(0, nnear, tile, ids, out.gj, part, lane, tg, c);
        adjoint_entries<T, V4, NB, false, RS>(nnear, len, tile, ids, out.gj, part, lane, tg, c);
        // FP32 tile partials of the four rows summed in FP64 (xor 16, xor 32)
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
            double px = kGScale * (double)fma_(tg.A[ib], tg.wx[ib], tg.Bx[ib]);
            double py = kGScale * (double)fma_(tg.A[ib], tg.wy[ib], tg.By[ib]);
            double pz = kGScale * (double)fma_(tg.A[ib], tg.wz[ib], tg.Bz[ib]);
            px += __shfl_xor(px, 16, 64);
            py += __shfl_xor(py, 16, 64);
            pz += __shfl_xor(pz, 16, 64);
            px += __shfl_xor(px, 32, 64);
            py += __shfl_xor(py, 32, 64);
            pz += __shfl_xor(pz, 32, 64);
            if (rb == ib) {
                gx -= px;
                gy -= py;
                gz -= pz;
            }
        }
    }
    if (lane < cnt) {
        out.gix[first + lane] = gx;
        out.giy[first + lane] = gy;
        out.giz[first + lane] = gz;
    }
}

template <class T, bool RS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_adjoint(GroupArgs ga, Src src, AdjCoef<T> c, const double* __restrict__ wx,
                                                const double* __restrict__ wy, const double* __restrict__ wz, int64_t ws,
                                                AdjOut out) {
    using V4 = typename Vec4<T>::type;
    __shared__ V4 tile[kTile + kRows];
    __shared__ int32_t ids[kTile + kRows];
    __shared__ T part[kGroupBlocks * kPartBlock];   // row partials of the j-side sums
    const int64_t g = xcd_block(blockIdx.x, gridDim.x);
    const int32_t first = ga.gfirst[g], cnt = ga.gcount[g];
    static_assert(kRow * kRows == 64, "one wave is kRows rows of kRow lanes");
    if (cnt > 48)
        adjoint_group<T, 4, RS>(ga, src, c, wx, wy, wz, ws, out, g, first, cnt, tile, ids, part);
    else if (cnt > 32)
        adjoint_group<T, 3, RS>(ga, src, c, wx, wy, wz, ws, out, g, first, cnt, tile, ids, part);
    else if (cnt > 16)
        adjoint_group<T, 2, RS>(ga, src, c, wx, wy, wz, ws, out, g, first, cnt, tile, ids, part);
    else
        adjoint_group<T, 1, RS>(ga, src, c, wx, wy, wz, ws, out, g, first, cnt, tile, ids, part);
}

// Node sources -> member particles.  For a cell c0 and its ancestors c
// (c0 included), with A_c = dL/dX_c / M_c:
//   SA(c0) = sum_c A_c,   T(c0) = sum_c [dL/dM_c + (X_c0 - X_c) . A_c].
// A particle k in leaf c0 then receives
//   dL/dx_k += m_k SA(c0),   dL/dm_k += T(c0) + (x_k - X_c0) . SA(c0),
// which equals sum_c [dL/dM_c + (x_k - X_c) . A_c] with every difference of
// positions formed before it is multiplied (no cancellation of large terms).
// Differences are taken to the nearest periodic image: a refitted cell's
// particles, and its centre of mass, may lie across a face of the unit box
// (the root, whose differences could reach half the box, is never a source).
__global__ void k_node_chain(int64_t nn, const NodeRange* __restrict__ rng, const double* __restrict__ M,
                             const double* __restrict__ X, const double* __restrict__ Y, const double* __restrict__ Z,
                             const double4* __restrict__ gn, double* __restrict__ sax, double* __restrict__ say,
                             double* __restrict__ saz, double* __restrict__ sb) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nn) return;
    const double x0 = X[c], y0 = Y[c], z0 = Z[c];
    double ax = 0, ay = 0, az = 0, b = 0;
    int32_t p = (int32_t)c;
    while (p >= 0) {
        const double inv = 1.0 / M[p];
        const double4 q = gn[p];
        const double a0 = q.x * inv, a1 = q.y * inv, a2 = q.z * inv;
        ax += a0;
        ay += a1;
        az += a2;
        b += q.w + (image(x0 - X[p]) * a0 + image(y0 - Y[p]) * a1 + image(z0 - Z[p]) * a2);
        p = rng[p].parent;
    }
    sax[c] = ax;
    say[c] = ay;
    saz[c] = az;
    sb[c] = b;
}

__global__ void k_adj_final(int64_t n, double G, const int32_t* __restrict__ perm, const int32_t* __restrict__ leaf_of,
                            const double* __restrict__ px, const double* __restrict__ py,
                            const double* __restrict__ pz, const double* __restrict__ pm,
                            const double* __restrict__ nX, const double* __restrict__ nY,
                            const double* __restrict__ nZ, AdjOut o, const double* __restrict__ sax,
                            const double* __restrict__ say, const double* __restrict__ saz,
                            const double* __restrict__ sb, double* __restrict__ gx, double* __restrict__ gy,
                            double* __restrict__ gz, int64_t gs, double* __restrict__ gm, int64_t gms) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t lf = leaf_of[s];
    const double a0 = sax[lf], a1 = say[lf], a2 = saz[lf], b = sb[lf];
    const double m = pm[s];
    const int64_t i = perm[s];
    const double4 gj = reinterpret_cast<const double4*>(o.gj)[s];
    gx[i * gs] = G * (o.gix[s] + gj.x + m * a0);
    gy[i * gs] = G * (o.giy[s] + gj.y + m * a1);
    gz[i * gs] = G * (o.giz[s] + gj.z + m * a2);
    gm[i * gms] = G * (gj.w + b + (image(px[s] - nX[lf]) * a0 + image(py[s] - nY[lf]) * a1 +
                                   image(pz[s] - nZ[lf]) * a2));
}

GroupArgs group_args(const Tree& t, const Lists& l) {
    GroupArgs ga;
    ga.gfirst = t.gfirst.get();
    ga.gcount = t.gcount.get();
    ga.glo = t.glo.get();
    ga.ghi = t.ghi.get();
    ga.off = l.off.get();
    ga.ent = l.ent.get();
    ga.perm = t.perm.get();
    return ga;
}

Src src_args(const Tree& t) {
    Src s;
    s.px = t.px.get();
    s.py = t.py.get();
    s.pz = t.pz.get();
    s.pm = t.pm.get();
    s.nX = t.nX.get();
    s.nY = t.nY.get();
    s.nZ = t.nZ.get();
    s.nM = t.nM.get();
    return s;
}

}  // namespace

// Far pairs of the FP32 kernels take r = s - eps^2/(2 s) (see far_r) when
// y = (2 eps / r_cut)^2 <= 5e-4, i.e. when its relative error y^2/8 stays
// below 3.2e-8, half an FP32 ulp.
static bool far_r_from_s(const srf_params& p) {
    const double y = 4.0 * p.eps * p.eps / (p.r_cut * p.r_cut);
    return y <= 5e-4;
}

void launch_force(const Tree& t, const Lists& l, const srf_params& p, double* ax, double* ay, double* az, int64_t os,
                  hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const int64_t ng = t.n_groups;
    if (ev0) SRF_HIP(hipEventRecord(ev0, st));
    if (p.precision == SRF_FP64) {
        hipLaunchKernelGGL((k_force<double, false, false>), dim3((unsigned)ng), dim3(64), 0, st, group_args(t, l),
                           src_args(t), make_coef<double>(p.r_cut, p.eps), p.G, ax, ay, az, os);
    } else {
        const bool rs = far_r_from_s(p);
        const Coef<float> c = make_coef<float>(p.r_cut, p.eps);
        const GroupArgs ga = group_args(t, l);
        const Src sa = src_args(t);
        if (p.compensated && rs)
            hipLaunchKernelGGL((k_force<float, true, true>), dim3((unsigned)ng), dim3(64), 0, st, ga, sa, c, p.G, ax,
                               ay, az, os);
        else if (p.compensated)
            hipLaunchKernelGGL((k_force<float, true, false>), dim3((unsigned)ng), dim3(64), 0, st, ga, sa, c, p.G, ax,
                               ay, az, os);
        else if (rs)
            hipLaunchKernelGGL((k_force<float, false, true>), dim3((unsigned)ng), dim3(64), 0, st, ga, sa, c, p.G, ax,
                               ay, az, os);
        else
            hipLaunchKernelGGL((k_force<float, false, false>), dim3((unsigned)ng), dim3(64), 0, st, ga, sa, c, p.G, ax,
                               ay, az, os);
    }
    SRF_HIP(hipGetLastError());
    if (ev1) SRF_HIP(hipEventRecord(ev1, st));
}

void launch_potential(const Tree& t, const Lists& l, const srf_params& p, double* phi, int64_t os, hipStream_t st) {
    const int64_t ng = t.n_groups;
    if (p.precision == SRF_FP64) {
        hipLaunchKernelGGL((k_potential<double, false>), dim3((unsigned)ng), dim3(64), 0, st, group_args(t, l),
                           src_args(t), make_pot_coef<double>(p.r_cut, p.eps), p.G, phi, os, (int32_t)t.n);
    } else if (far_r_from_s(p)) {
        hipLaunchKernelGGL((k_potential<float, true>), dim3((unsigned)ng), dim3(64), 0, st, group_args(t, l),
                           src_args(t), make_pot_coef<float>(p.r_cut, p.eps), p.G, phi, os, (int32_t)t.n);
    } else {
        hipLaunchKernelGGL((k_potential<float, false>), dim3((unsigned)ng), dim3(64), 0, st, group_args(t, l),
                           src_args(t), make_pot_coef<float>(p.r_cut, p.eps), p.G, phi, os, (int32_t)t.n);
    }
    SRF_HIP(hipGetLastError());
}

// Bytes of device workspace the adjoint needs: the j-side rows
// [n + n_cells][4], the i-side [3][n] and the cells' chain sums [4][n_cells]
// (FP64), each part starting on a 256-byte boundary.
static size_t adjoint_part_bytes(int64_t count) { return ((size_t)count * sizeof(double) + 255) & ~size_t(255); }

size_t adjoint_workspace_bytes(int64_t n, int64_t nn) {
    return adjoint_part_bytes(4 * (n + nn)) + adjoint_part_bytes(3 * n) + adjoint_part_bytes(4 * nn);
}

// The adjoint on a caller-provided workspace of adjoint_workspace_bytes()
// (256-byte aligned).  Its j-side rows are cleared here; the rest is written
// in full before it is read, so nothing of an earlier call leaks through.
static void adjoint_on(const Tree& t, const Lists& l, const srf_params& p, const double* wx, const double* wy,
                       const double* wz, int64_t ws, double* gx, double* gy, double* gz, int64_t gs, double* gm,
                       int64_t gms, void* work, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    const int64_t n = t.n, nn = t.n_nodes, ng = t.n_groups;
    char* w = static_cast<char*>(work);
    AdjOut o;
    o.gj = reinterpret_cast<double*>(w);          // [n + nn][4], 32-byte rows
    o.gn = o.gj + 4 * n;
    w += adjoint_part_bytes(4 * (n + nn));
    o.gix = reinterpret_cast<double*>(w);
    o.giy = o.gix + n;
    o.giz = o.giy + n;
    w += adjoint_part_bytes(3 * n);
    o.n = n;
    o.nn = nn;
    double* sax = reinterpret_cast<double*>(w);
    double* say = sax + nn;
    double* saz = say + nn;
    double* sb = saz + nn;
    fill_f64(o.gj, 0.0, 4 * (n + nn), st);
    if (ev0) SRF_HIP(hipEventRecord(ev0, st));
    if (p.precision == SRF_FP64) {
        hipLaunchKernelGGL((k_adjoint<double, false>), dim3((unsigned)ng), dim3(64), 0, st, group_args(t, l),
                           src_args(t), make_adj_coef<double>(p.r_cut, p.eps), wx, wy, wz, ws, o);
    } else if (far_r_from_s(p)) {
        hipLaunchKernelGGL((k_adjoint<float, true>), dim3((unsigned)ng), dim3(64), 0, st, group_args(t, l),
                           src_args(t), make_adj_coef<float>(p.r_cut, p.eps), wx, wy, wz, ws, o);
    } else {
        hipLaunchKernelGGL((k_adjoint<float, false>), dim3((unsigned)ng), dim3(64), 0, st, group_args(t, l),
                           src_args(t), make_adj_coef<float>(p.r_cut, p.eps), wx, wy, wz, ws, o);
    }
    SRF_HIP(hipGetLastError());
    if (ev1) SRF_HIP(hipEventRecord(ev1, st));
    hipLaunchKernelGGL(k_node_chain, dim3(grid_for(nn, 256, 1 << 30)), dim3(256), 0, st, nn, t.range.get(), t.nM.get(),
                       t.nX.get(), t.nY.get(), t.nZ.get(), reinterpret_cast<const double4*>(o.gn), sax, say, saz, sb);
    SRF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_adj_final, dim3(grid_for(n, 256, 1 << 30)), dim3(256), 0, st, n, p.G, t.perm.get(),
                       t.leaf_of.get(), t.px.get(), t.py.get(), t.pz.get(), t.pm.get(), t.nX.get(), t.nY.get(),
                       t.nZ.get(), o, sax, say, saz, sb, gx, gy, gz, gs, gm, gms);
    SRF_HIP(hipGetLastError());
}

void launch_adjoint(const Tree& t, const Lists& l, const srf_params& p, const double* wx, const double* wy,
                    const double* wz, int64_t ws, double* gx, double* gy, double* gz, int64_t gs, double* gm,
                    int64_t gms, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    DevBuf<char> work(adjoint_workspace_bytes(t.n, t.n_nodes), st);
    adjoint_on(t, l, p, wx, wy, wz, ws, gx, gy, gz, gs, gm, gms, work.get(), st, ev0, ev1);
}

// ------------------------------------------------- allocation-free adjoint
// The workspace of srf_short_range_adjoint_noalloc: a file-scope device
// array, one copy per GPU, held until the process ends.  Host code never
// passes the array's own name to a kernel (on the host it is only a stand-in
// for the symbol); it uses the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
static __device__ __align__(256) double scratch[SRF_NOALLOC_WORKSPACE_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_on_current_device() {
    int dev = 0;
    SRF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(SRF_EINVAL, "device index beyond the workspace table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        SRF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(SRF_EHIP, "hipGetSymbolAddress returned no address for the workspace");
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

void launch_adjoint_noalloc(const Tree& t, const Lists& l, const srf_params& p, const double* wx, const double* wy,
                            const double* wz, int64_t ws, double* gx, double* gy, double* gz, int64_t gs,
                            double* gm, int64_t gms, hipStream_t st) {
    const size_t need = adjoint_workspace_bytes(t.n, t.n_nodes);
    if (need > (size_t)SRF_NOALLOC_WORKSPACE_BYTES)
        fail(SRF_EINVAL, "the allocation-free adjoint needs " + std::to_string(need) +
                             " bytes of workspace for this tree; its static workspace holds " +
                             std::to_string((size_t)SRF_NOALLOC_WORKSPACE_BYTES));
    adjoint_on(t, l, p, wx, wy, wz, ws, gx, gy, gz, gs, gm, gms, scratch_on_current_device(), st, nullptr, nullptr);
}

}  // namespace srf
