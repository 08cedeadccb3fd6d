// jk_device.h -- device math and the two J/K kernel families for gfx950.
//
// Integral method: Rys quadrature (paper Section 2).  For a primitive
// quartet with exponents a, b, c, d on centres A, B, C, D, p = a + b,
// q = c + d, P and Q the Gaussian product centres and T = pq/(p+q)|PQ|^2:
//
//   (ab|cd) = 2 pi^(5/2) / (p q sqrt(p+q)) K_AB K_CD
//             sum_r w_r I_x(r) I_y(r) I_z(r)                       (eq. rys1)
//
// with N_r = floor((li+lj+lk+ll)/2) + 1 roots u_r = t_r^2 and weights w_r of
// the Rys polynomials of order N_r at T, and per-direction 2-D integrals
// I_x(a_x, b_x, c_x, d_x) (eq. rys2) built by the vertical recurrence
//
//   G(n+1, m) = C00 G(n, m) + n B10 G(n-1, m) + m B00 G(n, m-1)
//   G(n, m+1) = C00' G(n, m) + m B01 G(n, m-1) + n B00 G(n-1, m)
//   B00 = u / (2(p+q)),  B10 = (1 - q u/(p+q)) / (2p),  B01 = (1 - p u/(p+q)) / (2q)
//   C00 = (P - A) - q u/(p+q) (P - Q),  C00' = (Q - C) + p u/(p+q) (P - Q)
//
// then horizontal transfer I(a, b+1) = I(a+1, b) + (A - B) I(a, b) on the
// bra and likewise with (C - D) on the ket.
//
// J/K digestion (Section 2, eq. jk, over unique quartets): a unique shell
// quartet with degeneracy weight w = 2^-[I=J] 2^-[K=L] 2^-[IJ=KL] feeds
//   J'_ab += 2w v D_cd,  J'_cd += 2w v D_ab,
//   K'_ac += w v D_bd,  K'_ad += w v D_bc,  K'_bc += w v D_ad,  K'_bd += w v D_ac,
// and J = J' + J'^T, K = K' + K'^T afterwards (finalize kernel).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jk_common.h"
#include "tables/jk_tables_meta.h"
#include "tables/jk_tables_mom_meta.h"

namespace jk {

constexpr double TWO_PI_2_5 = 34.986836655249725;  // 2 pi^(5/2)
constexpr double SQRT_PI_HALF = 0.88622692545275801;  // sqrt(pi) / 2

// Reciprocal and reciprocal square root: hardware estimate refined by two
// Newton steps in FP64 (each step doubles the correct bits), hardware
// instruction alone in FP32.  Arguments are positive and finite here.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}
__device__ __forceinline__ double rsq64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}
template <typename R> __device__ __forceinline__ R rsqrt_(R x);
template <> __device__ __forceinline__ double rsqrt_<double>(double x) { return rsq64(x); }
template <> __device__ __forceinline__ float rsqrt_<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <typename R> __device__ __forceinline__ R rcp_(R x);
template <> __device__ __forceinline__ double rcp_<double>(double x) { return rcp64(x); }
template <> __device__ __forceinline__ float rcp_<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R> struct TabSel;
template <> struct TabSel<double> {
    static __device__ __forceinline__ const double *rys(const Tables &t) { return t.rys; }
    static __device__ __forceinline__ const double *hx2(const Tables &t) { return t.hx2; }
    static __device__ __forceinline__ const double *hw(const Tables &t) { return t.hw; }
    static __device__ __forceinline__ const double *boys(const Tables &t) { return t.boys; }
};
template <> struct TabSel<float> {
    static __device__ __forceinline__ const float *rys(const Tables &t) { return t.rys32; }
    static __device__ __forceinline__ const float *hx2(const Tables &t) { return t.hx2_32; }
    static __device__ __forceinline__ const float *hw(const Tables &t) { return t.hw32; }
    static __device__ __forceinline__ const float *boys(const Tables &t) { return t.boys32; }
};

// ---------------------------------------------------------------------------
// One-root case: u = F_1 / F_0, w = F_0 from the tabulated Boys function.
// Below the table end both come from the Taylor expansion about the nearest
// grid point T_j (spacing 1/32), F_m(T) = sum_k F_(m+k)(T_j) (T_j - T)^k / k!,
// 7 terms in FP64 and 4 in FP32 (no exponential needed).  Above it, the
// large-T limits F_0 = sqrt(pi/T) / 2 and F_1 = F_0 / (2T), evaluated in FP64
// in both precisions.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void rys1(double T, const R *__restrict__ boys, R &u, R &w) {
    if (T < JKT_BOYS_TMAX) {
        const int j = (int)(T * JKT_BOYS_DENSITY + 0.5);
        const R d = (R)((double)j * (1.0 / JKT_BOYS_DENSITY) - T);  // T_j - T
        const R *row = boys + j * (JKT_BOYS_MMAX + 1);
        constexpr int NT = sizeof(R) == 8 ? 7 : 4;  // Taylor terms
        // d / k once for both expansions (each Horner step is then one FMA)
        R dk[NT];
#pragma unroll
        for (int k = 1; k < NT; ++k) dk[k] = d * (R)(1.0 / k);
        R f1 = row[NT];
        R f0 = row[NT - 1];
#pragma unroll
        for (int k = NT - 1; k >= 1; --k) {
            f1 = row[k] + f1 * dk[k];
            f0 = row[k - 1] + f0 * dk[k];
        }
        w = f0;
        u = f1 * rcp_<R>(f0);
    } else {
        // large T: the asymptotic Boys values, in FP64 for both precisions
        const double rt = rsq64(T);
        w = (R)(SQRT_PI_HALF * rt);
        u = (R)(0.5 * rt * rt);
    }
}

// The same rule in two stages, so that the grid row of the next primitive
// quartet can be in flight while the current one is evaluated: rys1_fetch
// loads the row (lanes beyond the table end load nothing and leave the row
// as it was: rys1_eval does not read it for them) and rys1_eval gives
// exactly the values of rys1.
template <typename R>
struct Rys1Row {
    static constexpr int NT = sizeof(R) == 8 ? 7 : 4;  // Taylor terms
    R f[NT + 1];
    R d;  // T_j - T
};
template <typename R>
__device__ __forceinline__ void rys1_fetch(double T, const R *__restrict__ boys, Rys1Row<R> &row) {
    if (T < JKT_BOYS_TMAX) {
        const int j = (int)(T * JKT_BOYS_DENSITY + 0.5);
        row.d = (R)((double)j * (1.0 / JKT_BOYS_DENSITY) - T);
        const R *src = boys + j * (JKT_BOYS_MMAX + 1);
#pragma unroll
        for (int k = 0; k <= Rys1Row<R>::NT; ++k) row.f[k] = src[k];
    }
}
template <typename R>
__device__ __forceinline__ void rys1_eval(double T, const Rys1Row<R> &row, R &u, R &w) {
    constexpr int NT = Rys1Row<R>::NT;
    if (T < JKT_BOYS_TMAX) {
        const R d = row.d;
        // d / k once for both expansions (each Horner step is then one FMA)
        R dk[NT];
#pragma unroll
        for (int k = 1; k < NT; ++k) dk[k] = d * (R)(1.0 / k);
        R f1 = row.f[NT];
        R f0 = row.f[NT - 1];
#pragma unroll
        for (int k = NT - 1; k >= 1; --k) {
            f1 = row.f[k] + f1 * dk[k];
            f0 = row.f[k - 1] + f0 * dk[k];
        }
        w = f0;
        u = f1 * rcp_<R>(f0);
    } else {
        // large T: the asymptotic Boys values, in FP64 for both precisions
        const double rt = rsq64(T);
        w = (R)(SQRT_PI_HALF * rt);
        u = (R)(0.5 * rt * rt);
    }
}

// ---------------------------------------------------------------------------
// Two roots in FP64 from the moments F_0..F_3 (the defining property of the
// rule: sum_i w_i u_i^k = F_k(T) for k = 0..3).  F_3 and e^-T are expanded
// about the nearest grid point T_j (7 Taylor terms each, |T_j - T| <= 1/64),
// F_2, F_1, F_0 follow by the stable downward recursion
// F_m = (2T F_(m+1) + e^-T) / (2m+1).  The nodes are the zeros of the
// monic orthogonal polynomial u^2 + a u + b with
//   F_2 + a F_1 + b F_0 = 0,  F_3 + a F_2 + b F_1 = 0,
// taken as u_+ = (-a + sqrt(a^2 - 4b)) / 2 and u_- = b / u_+ (no
// cancellation since a < 0), with weights w_+ = (F_1 - u_- F_0) / (u_+ - u_-)
// and w_- = F_0 - w_+.  Beyond the grid: the Gauss-Hermite limit.  One row
// of 64 bytes per primitive quartet instead of the fit coefficients.
// ---------------------------------------------------------------------------
struct Rys2Row {
    double f[JKT_MOM_COLS];  // e^-T_j, F_3(T_j) .. F_9(T_j)
    double d;                // T_j - T
};
static_assert(JKT_MOM_M0 == 3 && JKT_MOM_COLS == JKT_MOM_TERMS + 1, "moment grid layout");

__device__ __forceinline__ void rys2_fetch(double T, const double *__restrict__ mom, Rys2Row &row) {
    if (T < JKT_MOM_TMAX) {
        const int j = (int)(T * JKT_MOM_DENSITY + 0.5);
        row.d = (double)j * (1.0 / JKT_MOM_DENSITY) - T;
        const double *src = mom + j * JKT_MOM_COLS;
#pragma unroll
        for (int k = 0; k < JKT_MOM_COLS; ++k) row.f[k] = src[k];
    }
    // (beyond the grid the row keeps its contents: rys2_eval does not read it)
}

__device__ __forceinline__ void rys2_eval(double T, const Rys2Row &row, double (&u)[2], double (&w)[2]) {
    if (T < JKT_MOM_TMAX) {
        const double d = row.d;
        double f3 = row.f[JKT_MOM_TERMS];
        double ed = 1.0;
#pragma unroll
        for (int k = JKT_MOM_TERMS - 1; k >= 1; --k) {
            f3 = row.f[k] + f3 * d * (1.0 / k);
            ed = 1.0 + ed * d * (1.0 / k);
        }
        const double ex = row.f[0] * ed;
        const double t2 = T + T;
        const double f2 = (t2 * f3 + ex) * (1.0 / 5.0);
        const double f1 = (t2 * f2 + ex) * (1.0 / 3.0);
        const double f0 = t2 * f1 + ex;
        const double rdet = rcp64(f1 * f1 - f0 * f2);
        const double a = (f0 * f3 - f1 * f2) * rdet;
        const double b = (f2 * f2 - f1 * f3) * rdet;
        const double disc = a * a - 4.0 * b;
        const double up = 0.5 * (disc * rsq64(disc) - a);
        const double um = b * rcp64(up);
        const double wp = (f1 - um * f0) * rcp64(up - um);
        u[0] = um;
        u[1] = up;
        w[0] = f0 - wp;
        w[1] = wp;
    } else {
        const double rt = rsq64(T);
        const double rT = rt * rt;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            u[i] = jkt_mom_hx2[i] * rT;
            w[i] = jkt_mom_hw[i] * rt;
        }
    }
}

// ---------------------------------------------------------------------------
// N >= 2 roots: piecewise polynomial fits on unit intervals of T (Horner on
// all 2N functions at once, degree-major layout), large-T Gauss-Hermite limit.
// ---------------------------------------------------------------------------
template <int N, typename R>
__device__ __forceinline__ void rys_roots(double T, const Tables &tab, R (&u)[N], R (&w)[N]) {
    if constexpr (N == 1) {
        rys1<R>(T, TabSel<R>::boys(tab), u[0], w[0]);
    } else if constexpr (N == 2) {
        // FP64 for both precisions (single-precision kernels round it)
        Rys2Row row;
        rys2_fetch(T, tab.mom, row);
        double ud[2], wd[2];
        rys2_eval(T, row, ud, wd);
        u[0] = (R)ud[0]; u[1] = (R)ud[1];
        w[0] = (R)wd[0]; w[1] = (R)wd[1];
    } else {
        static_assert(jkt_rys_h[N] == 1.0, "unit intervals assumed");
        constexpr int NF = 2 * N;
        if (T < jkt_rys_tmax[N]) {
            const int it = (int)T;
            const R x = (R)(2.0 * (T - (double)it) - 1.0);
            const R *c = TabSel<R>::rys(tab) + jkt_rys_offset[N] + (it * (JKT_RYS_DEG + 1) + JKT_RYS_DEG) * NF;
            R acc[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f] = c[f];
#pragma unroll
            for (int k = JKT_RYS_DEG - 1; k >= 0; --k) {
                c -= NF;
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f] = acc[f] * x + c[f];
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                u[i] = acc[i];
                w[i] = acc[N + i];
            }
        } else {
            // large T: the Gauss-Hermite limit, in FP64 for both precisions
            const double rt = rsq64(T);
            const double rT = rt * rt;
            const double *hx = tab.hx2 + jkt_herm_offset[N];
            const double *hw = tab.hw + jkt_herm_offset[N];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                u[i] = (R)(hx[i] * rT);
                w[i] = (R)(hw[i] * rt);
            }
        }
    }
}

// Root rules evaluated in two stages (the table row of one primitive
// quartet is loaded while the previous one is evaluated): one and two roots.
template <int N, typename R>
struct RootPipe {
    static constexpr bool ok = false;
};
template <typename R>
struct RootPipe<1, R> {
    static constexpr bool ok = true;
    using Row = Rys1Row<R>;
    static __device__ __forceinline__ void fetch(double T, const Tables &tab, Row &row) {
        rys1_fetch<R>(T, TabSel<R>::boys(tab), row);
    }
    static __device__ __forceinline__ void eval(double T, const Row &row, const Tables &, R (&u)[1], R (&w)[1]) {
        rys1_eval<R>(T, row, u[0], w[0]);
    }
};
template <typename R>
struct RootPipe<2, R> {
    static constexpr bool ok = true;
    using Row = Rys2Row;
    static __device__ __forceinline__ void fetch(double T, const Tables &tab, Row &row) { rys2_fetch(T, tab.mom, row); }
    static __device__ __forceinline__ void eval(double T, const Row &row, const Tables &, R (&u)[2], R (&w)[2]) {
        double ud[2], wd[2];
        rys2_eval(T, row, ud, wd);
        u[0] = (R)ud[0]; u[1] = (R)ud[1];
        w[0] = (R)wd[0]; w[1] = (R)wd[1];
    }
};

// single root r of an N-root rule (the 2-D table builders of family 2)
template <int N, typename R>
__device__ __forceinline__ void rys_root1(double T, int r, const Tables &tab, R &u, R &w) {
    if constexpr (N == 1) {
        rys1<R>(T, TabSel<R>::boys(tab), u, w);
    } else {
        constexpr int NF = 2 * N;
        if (T < jkt_rys_tmax[N]) {
            const int it = (int)T;
            const R x = (R)(2.0 * (T - (double)it) - 1.0);
            const R *c = TabSel<R>::rys(tab) + jkt_rys_offset[N] + (it * (JKT_RYS_DEG + 1) + JKT_RYS_DEG) * NF;
            R au = c[r], aw = c[N + r];
#pragma unroll
            for (int k = JKT_RYS_DEG - 1; k >= 0; --k) {
                c -= NF;
                au = au * x + c[r];
                aw = aw * x + c[N + r];
            }
            u = au;
            w = aw;
        } else {
            // large T: the Gauss-Hermite limit, in FP64 for both precisions
            const double rt = rsq64(T);
            u = (R)(tab.hx2[jkt_herm_offset[N] + r] * rt * rt);
            w = (R)(tab.hw[jkt_herm_offset[N] + r] * rt);
        }
    }
}

// ---------------------------------------------------------------------------
// Range separation (the range-separation parameter omega).  The integrand of
// the long-range operator erf(omega r)/r is the Coulomb one restricted to
// t in [0, theta], theta^2 = omega^2 / (omega^2 + rho): substituting t =
// theta s turns it into a standard Rys rule at theta^2 T whose roots t^2 are
// theta^2 times the standard roots and whose weights carry a factor theta.
// The short-range operator erfc(|omega| r)/r is the full one minus the long
// one.  A primitive quartet is therefore evaluated as one or two "variants":
//   omega = 0: variant 0 (full range);  omega > 0: variant 1 (long range);
//   omega < 0: variant 0 plus variant 1 with negated weights.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int variant_begin(double omega) { return omega > 0.0 ? 1 : 0; }
__device__ __forceinline__ int variant_end(double omega) { return omega == 0.0 ? 1 : 2; }

template <int N, typename R>
__device__ __forceinline__ void rys_roots_op(double T, double rho, double omega, int variant, const Tables &tab,
                                             R (&u)[N], R (&w)[N]) {
    if (variant == 0) {
        rys_roots<N, R>(T, tab, u, w);
        return;
    }
    const double w2 = omega * omega, th2 = w2 / (w2 + rho);
    rys_roots<N, R>(th2 * T, tab, u, w);
    const double th = sqrt(th2);
    const R su = (R)th2, sw = (R)(omega > 0.0 ? th : -th);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        u[i] *= su;
        w[i] *= sw;
    }
}

template <int N, typename R>
__device__ __forceinline__ void rys_root1_op(double T, double rho, double omega, int variant, int r,
                                             const Tables &tab, R &u, R &w) {
    if (variant == 0) {
        rys_root1<N, R>(T, r, tab, u, w);
        return;
    }
    const double w2 = omega * omega, th2 = w2 / (w2 + rho);
    rys_root1<N, R>(th2 * T, r, tab, u, w);
    const double th = sqrt(th2);
    u *= (R)th2;
    w *= (R)(omega > 0.0 ? th : -th);
}

// ---------------------------------------------------------------------------
// 2-D integrals of one direction for one root: vertical recurrence G(n, m)
// scaled by s, then horizontal transfers; emit(a, b, c, d, value) receives
// every I(a, b, c, d), a <= LI, b <= LJ, c <= LK, d <= LL, in b-major order.
// ---------------------------------------------------------------------------
template <int LI, int LJ, int LK, int LL, typename R, typename Emit>
__device__ __forceinline__ void rys2d(R c00, R c00p, R b00, R b10, R b01, R ab, R cd, R s, Emit &&emit) {
    constexpr int NA = LI + LJ, NC = LK + LL;
    R G[NA + 1][NC + 1];
    G[0][0] = s;
    if constexpr (NA > 0) G[1][0] = c00 * s;
#pragma unroll
    for (int n = 1; n < NA; ++n) G[n + 1][0] = c00 * G[n][0] + (R)n * b10 * G[n - 1][0];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
#pragma unroll
        for (int n = 0; n <= NA; ++n) {
            R v = c00p * G[n][m];
            if (m > 0) v += (R)m * b01 * G[n][m - 1];
            if (n > 0) v += (R)n * b00 * G[n - 1][m];
            G[n][m + 1] = v;
        }
    }
    // bra transfer, one b level at a time; X[a][m] holds level b for a <= NA - b
    R X[NA + 1][NC + 1];
#pragma unroll
    for (int n = 0; n <= NA; ++n)
#pragma unroll
        for (int m = 0; m <= NC; ++m) X[n][m] = G[n][m];
#pragma unroll
    for (int b = 0; b <= LJ; ++b) {
        if (b > 0) {
#pragma unroll
            for (int n = 0; n <= NA - b; ++n)
#pragma unroll
                for (int m = 0; m <= NC; ++m) X[n][m] = X[n + 1][m] + ab * X[n][m];
        }
#pragma unroll
        for (int a = 0; a <= LI; ++a) {
            // ket transfer on X[a][0..NC]
            R Y[NC + 1];
#pragma unroll
            for (int m = 0; m <= NC; ++m) Y[m] = X[a][m];
#pragma unroll
            for (int d = 0; d <= LL; ++d) {
                if (d > 0) {
#pragma unroll
                    for (int c = 0; c <= NC - d; ++c) Y[c] = Y[c + 1] + cd * Y[c];
                }
#pragma unroll
                for (int c = 0; c <= LK; ++c) emit(a, b, c, d, Y[c]);
            }
        }
    }
}

template <int LI, int LJ, int LK, int LL>
struct Cls {
    static constexpr int NI = ncart(LI), NJ = ncart(LJ), NK = ncart(LK), NL = ncart(LL);
    static constexpr int NAB = NI * NJ, NCD = NK * NL, NC = NAB * NCD;
    static constexpr int NR = nroots(LI, LJ, LK, LL);
    static constexpr int S = (LI + 1) * (LJ + 1) * (LK + 1) * (LL + 1);
    // index of I(a, b, c, d) in a [a][b][c][d] table
    static __device__ __forceinline__ constexpr int t4(int a, int b, int c, int d) {
        return ((a * (LJ + 1) + b) * (LK + 1) + c) * (LL + 1) + d;
    }
};

// Lane index within the wave.  Taken from threadIdx rather than mbcnt:
// mbcnt counts the active lanes below the current one, which differs from
// the lane index when the compiler evaluates it under a partial EXEC mask.
__device__ __forceinline__ int lane_index() { return (int)(threadIdx.x & 63u); }

// Orders a wave's LDS writes before its later LDS reads by other lanes of
// the same wave (the LDS tables of family 2 are private to one wave, so no
// workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ void atomic_add_f64(double *p, T v) {
    unsafeAtomicAdd(p, (double)v);
}

// Fixed-order accumulation.  v is split exactly into integer multiples of
// 2^-16 and 2^-56 and a multiple of 2^-96 rounded to nearest (each below
// 2^40 in magnitude for |v| < 2^24), and each part is added to its own
// 64-bit integer limb, L elements apart.  Integer additions commute, so the
// limbs end the same whatever order the additions came in, for up to 2^23
// additions per element; k_det_collapse then forms the double in a fixed
// order.
__device__ __forceinline__ void det_add(double *p, int64_t L, double v) {
    if (v == 0.0) return;
    unsigned long long *q = reinterpret_cast<unsigned long long *>(p);
    const double x0 = v * 0x1p16;
    const double t0 = trunc(x0);
    const double x1 = (x0 - t0) * 0x1p40;
    const double t1 = trunc(x1);
    const double t2 = rint((x1 - t1) * 0x1p40);
    if (t0 != 0.0) atomicAdd(q, (unsigned long long)(long long)t0);
    if (t1 != 0.0) atomicAdd(q + L, (unsigned long long)(long long)t1);
    if (t2 != 0.0) atomicAdd(q + 2 * L, (unsigned long long)(long long)t2);
}
// A tile kernel's addition into J, K or the pair-ordered J' buffer.
template <typename T>
__device__ __forceinline__ void acc_add(const JkArgs &a, double *p, T v) {
    if (a.det) det_add(p, a.det, (double)v);
    else atomic_add_f64(p, v);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Largest i in [0, n) with off[i] <= key (off ascending, off[0] = 0).
__device__ __forceinline__ int tile_bra(const int32_t *__restrict__ off, int n, int key) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double dmax6(const JkArgs &a, const PairRec &B, const PairRec &K) {
    const double *dm = a.dmax;
    const int n = a.nshell;
    double m = dm[B.ish * n + B.jsh];
    m = fmax(m, dm[K.ish * n + K.jsh]);
    m = fmax(m, dm[B.ish * n + K.ish]);
    m = fmax(m, dm[B.ish * n + K.jsh]);
    m = fmax(m, dm[B.jsh * n + K.ish]);
    m = fmax(m, dm[B.jsh * n + K.jsh]);
    return m;
}

// Screening and precision split of one quartet from its bound
// Q_IJ Q_KL max|D| over the six blocks it touches (FP64): below dscreen
// (> 0) the quartet is dropped (density screening); the single-precision
// pass of the mixed split keeps the quartets below mix_thr, the
// double-precision pass those at or above it.  Both settings are uniform in
// the launch, so the branch on them is too.
__device__ __forceinline__ void screen_quartet(const JkArgs &a, const PairRec &B, const PairRec &K, bool &valid) {
    if (a.dscreen > 0.0 || a.sel != SEL_ALL) {
        const double bound = B.q * K.q * dmax6(a, B, K);
        if (a.dscreen > 0.0) valid = valid && bound >= a.dscreen;
        if (a.sel == SEL_LO) valid = valid && bound < a.mix_thr;
        else if (a.sel == SEL_HI) valid = valid && bound >= a.mix_thr;
    }
}

// Whether any quartet of a bra with Schwarz factor qb and a ket with factor
// at most qk can still be selected, from the largest density block of all:
// the ket lists are sorted by Schwarz factor (descending), so once this
// fails for the first ket of a chunk it fails for every later ket of the bra
// (the double-precision pass of the mixed split, density screening).
__device__ __forceinline__ bool prefix_selectable(const JkArgs &a, double qb, double qk) {
    if (a.sel != SEL_HI && a.dscreen <= 0.0) return true;
    const double b = qb * qk * a.dmax[a.nshell * a.nshell];
    return (a.sel != SEL_HI || b >= a.mix_thr) && (a.dscreen <= 0.0 || b >= a.dscreen);
}

// Number of a wave's lanes with mine set (one lane per quartet): the
// quartets the wave evaluates; a wave with none skips the work as a whole.
__device__ __forceinline__ int count_selected(bool mine) { return (int)__popcll(__ballot(mine)); }

// Adds a wave's evaluated quartets to the launch's counters (one atomic from
// one lane; the slot follows the workgroup).
__device__ __forceinline__ void add_count(const JkArgs &a, int n) {
    if (a.nsel && n > 0 && lane_index() == 0)
        atomicAdd(&a.nsel[(blockIdx.x % NSEL_SLOTS) * NSEL_STRIDE], (unsigned long long)n);
}

__device__ __forceinline__ double pair_weight(int bra, int ket, const PairRec &B, const PairRec &K) {
    double w = 1.0;
    if (B.ish == B.jsh) w *= 0.5;
    if (K.ish == K.jsh) w *= 0.5;
    if (bra == ket) w *= 0.5;
    return w;
}

// Geometry of one primitive quartet.  Differences of centres are formed in
// FP64 and rounded to R afterwards.
template <typename R>
struct PQuart {
    double T, rho;  // T = rho |PQ|^2, rho = pq / (p + q)
    R fq, fp, rpq, pref, hb, hk;
    R PQ[3], PA[3], QC[3];
};

// First stage of a primitive quartet's geometry: 1/sqrt(p+q), rho and T
// (what the root table lookup needs); prim_rest finishes the quartet.
template <typename R>
struct PT {
    double T, rho;
    R rs;  // 1 / sqrt(p + q)
};

template <typename R>
__device__ __forceinline__ PT<R> prim_T(const PrimPair &pb, const PrimPair &pk) {
    PT<R> t;
    if constexpr (sizeof(R) == 4) {
        // single precision quartets: only the centre differences and the
        // prefactor's product of pair factors are formed in FP64
        const float p = (float)pb.p, q = (float)pk.p;
        const float rs = __builtin_amdgcn_rsqf(p + q);
        const float rpq = rs * rs;
        float pq2 = 0.0f;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const float d = (float)(pb.P[x] - pk.P[x]);
            pq2 += d * d;
        }
        const float rho = p * q * rpq;
        t.rho = (double)rho;
        t.T = (double)(rho * pq2);
        t.rs = rs;
    } else {
        const double p = pb.p, q = pk.p;
        const double rs = rsq64(p + q);
        const double rpq = rs * rs;
        double pq2 = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const double d = pb.P[x] - pk.P[x];
            pq2 += d * d;
        }
        t.rho = p * q * rpq;
        t.T = t.rho * pq2;
        t.rs = rs;
    }
    return t;
}

template <typename R>
__device__ __forceinline__ PQuart<R> prim_rest(const PrimPair &pb, const PrimPair &pk, const PT<R> &t) {
    PQuart<R> g;
    g.T = t.T;
    g.rho = t.rho;
    const R rs = t.rs, rpq = rs * rs;
    g.rpq = rpq;
    g.fq = (R)pk.p * rpq;
    g.fp = (R)pb.p * rpq;
    if constexpr (sizeof(R) == 4) g.pref = (float)(TWO_PI_2_5 * pb.kp * pk.kp) * rs;
    else g.pref = TWO_PI_2_5 * pb.kp * pk.kp * rs;
    g.hb = (R)pb.h;
    g.hk = (R)pk.h;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        g.PQ[x] = (R)(pb.P[x] - pk.P[x]);
        g.PA[x] = (R)pb.PA[x];
        g.QC[x] = (R)pk.PA[x];
    }
    return g;
}

template <typename R>
__device__ __forceinline__ PQuart<R> prim_quartet(const PrimPair &pb, const PrimPair &pk) {
    return prim_rest<R>(pb, pk, prim_T<R>(pb, pk));
}

// ===========================================================================
// Family 1: one lane per quartet.  The contracted Cartesian block V lives in
// registers; digestion reduces J_IJ across the wave when the bra is uniform
// (tiles), adds J_KL into the pair-ordered buffer and sends the K blocks
// straight to FP64 atomics.
// ===========================================================================
// Waits for the loads of a record here, once: values that are still
// loading at the top of a loop make the compiler wait for every load issued
// since (here: the next quartet's root table row) wherever they are used.
__device__ __forceinline__ void settle(double &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void settle(float &x) { asm volatile("" : "+v"(x)); }
// one of three values by index, as selects on opaque registers
template <typename R>
__device__ __forceinline__ R sel3(int x, R v0, R v1, R v2) {
    settle(v0);
    settle(v1);
    settle(v2);
    return x == 0 ? v0 : (x == 1 ? v1 : v2);
}
__device__ __forceinline__ void settle(PrimPair &r) {
    settle(r.p);
    settle(r.h);
    settle(r.kp);
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        settle(r.P[x]);
        settle(r.PA[x]);
    }
}

// Adds the N_r roots of one primitive quartet to the contracted block V.
template <int LI, int LJ, int LK, int LL, typename R>
__device__ __forceinline__ void k1_roots_acc(const PQuart<R> &g, const R *u, const R *w, const R (&ab)[3],
                                             const R (&cd)[3], R (&V)[ncart4(LI, LJ, LK, LL)]) {
    using C = Cls<LI, LJ, LK, LL>;
    constexpr int NI = C::NI, NJ = C::NJ, NK = C::NK, NL = C::NL, NR = C::NR;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const R t = u[r];
        const R b00 = (R)0.5 * t * g.rpq;
        const R b10 = g.hb * ((R)1 - g.fq * t);
        const R b01 = g.hk * ((R)1 - g.fp * t);
        R I[3][C::S];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const R c00 = g.PA[x] - g.fq * t * g.PQ[x];
            const R c00p = g.QC[x] + g.fp * t * g.PQ[x];
            const R s = x == 2 ? w[r] * g.pref : (R)1;
            R *dst = I[x];
            rys2d<LI, LJ, LK, LL, R>(c00, c00p, b00, b10, b01, ab[x], cd[x], s,
                                     [&](int ia, int ib2, int ic, int id, R v) { dst[C::t4(ia, ib2, ic, id)] = v; });
        }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int k = 0; k < NK; ++k)
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        const int ix = C::t4(cart_comp(LI, i, 0), cart_comp(LJ, j, 0), cart_comp(LK, k, 0), cart_comp(LL, l, 0));
                        const int iy = C::t4(cart_comp(LI, i, 1), cart_comp(LJ, j, 1), cart_comp(LK, k, 1), cart_comp(LL, l, 1));
                        const int iz = C::t4(cart_comp(LI, i, 2), cart_comp(LJ, j, 2), cart_comp(LK, k, 2), cart_comp(LL, l, 2));
                        V[((i * NJ + j) * NK + k) * NL + l] += I[0][ix] * I[1][iy] * I[2][iz];
                    }
    }
}

// Contracted Cartesian block of one quartet into V (registers); pbat(ib)
// returns the bra's primitive pair record ib.  RS: the range-separated
// operators (omega != 0) are compiled in; the Coulomb instance has no
// trace of them (given the chance, the compiler evaluates the root scaling
// of the other variant on every primitive quartet).
template <int LI, int LJ, int LK, int LL, typename R, bool RS, typename PBF>
__device__ __forceinline__ void k1_compute_op(const JkArgs &a, const PairRec &B, const PairRec &Kt, PBF &&pbat, int npb,
                                              int npk, R (&V)[ncart4(LI, LJ, LK, LL)]) {
    using C = Cls<LI, LJ, LK, LL>;
    constexpr int NR = C::NR;
#pragma unroll
    for (int e = 0; e < C::NC; ++e) V[e] = (R)0;
    const R ab[3] = {(R)B.ab[0], (R)B.ab[1], (R)B.ab[2]};
    const R cd[3] = {(R)Kt.ab[0], (R)Kt.ab[1], (R)Kt.ab[2]};
    // ket primitive outer (one vector load each), bra primitive inner (the
    // bra is uniform across a tile or row task)
    if constexpr (!RS && RootPipe<NR, R>::ok) {
        // the root table row of the next primitive quartet is loaded while
        // the current one's recurrences run
        using P = RootPipe<NR, R>;
        // the next ket primitive's record loads while the current one's bra
        // primitives run
        // (the one-root classes load each ket record when they reach it:
        // their registers, not the load, bound them)
        constexpr bool PREF = NR > 1;
        PrimPair pk = a.pp[Kt.pp_off];
        settle(pk);
        for (int ik = 0; ik < npk; ++ik) {
            PrimPair pkn;
            if (PREF && ik + 1 < npk) pkn = a.pp[Kt.pp_off + (ik + 1) * Kt.pp_stride];
            PT<R> t = prim_T<R>(pbat(0), pk);
            typename P::Row row;
            P::fetch(t.T, a.tab, row);
            for (int ib = 0; ib < npb; ++ib) {
                const PQuart<R> g = prim_rest<R>(pbat(ib), pk, t);
                R u[NR], w[NR];
                P::eval(g.T, row, a.tab, u, w);
                if (ib + 1 < npb) {
                    t = prim_T<R>(pbat(ib + 1), pk);
                    P::fetch(t.T, a.tab, row);
                }
                k1_roots_acc<LI, LJ, LK, LL, R>(g, u, w, ab, cd, V);
            }
            if (ik + 1 < npk) {
                if constexpr (PREF) {
                    settle(pkn);
                    pk = pkn;
                } else {
                    pk = a.pp[Kt.pp_off + (ik + 1) * Kt.pp_stride];
                }
            }
        }
        return;
    }
    const int vb = RS ? variant_begin(a.omega) : 0, ve = RS ? variant_end(a.omega) : 1;
    for (int ik = 0; ik < npk; ++ik) {
        const PrimPair pk = a.pp[Kt.pp_off + ik * Kt.pp_stride];
        for (int ib = 0; ib < npb; ++ib) {
            const PQuart<R> g = prim_quartet<R>(pbat(ib), pk);
            for (int var = vb; var < ve; ++var) {
                R u[NR], w[NR];
                if constexpr (RS) rys_roots_op<NR, R>(g.T, g.rho, a.omega, var, a.tab, u, w);
                else rys_roots<NR, R>(g.T, a.tab, u, w);
                k1_roots_acc<LI, LJ, LK, LL, R>(g, u, w, ab, cd, V);
            }
        }
    }
}

template <int LI, int LJ, int LK, int LL, typename R, typename PBF>
__device__ __forceinline__ void k1_compute(const JkArgs &a, const PairRec &B, const PairRec &Kt, PBF &&pbat, int npb,
                                           int npk, R (&V)[ncart4(LI, LJ, LK, LL)]) {
    if (a.omega == 0.0) k1_compute_op<LI, LJ, LK, LL, R, false>(a, B, Kt, pbat, npb, npk, V);
    else k1_compute_op<LI, LJ, LK, LL, R, true>(a, B, Kt, pbat, npb, npk, V);
}

template <int LI, int LJ, int LK, int LL, typename R, int MODE>
__device__ __forceinline__ void k1_body(const JkArgs &a, int bra, int ket, bool valid, double wq, int64_t gout) {
    using C = Cls<LI, LJ, LK, LL>;
    constexpr int NI = C::NI, NJ = C::NJ, NK = C::NK, NL = C::NL, NAB = C::NAB, NCD = C::NCD;
    constexpr bool BRA_UNIFORM = MODE == MODE_JK;
    const int lane = lane_index();
    const PairRec B = a.pairs[bra];
    const PairRec Kt = a.pairs[ket];
    R V[C::NC];
    k1_compute<LI, LJ, LK, LL, R>(a, B, Kt, [&](int ib) { return a.pp[B.pp_off + ib * B.pp_stride]; },
                                  BRA_UNIFORM ? a.npb : B.npp, MODE == MODE_JK ? a.npk : Kt.npp, V);
    if constexpr (MODE == MODE_EXPORT) {
        if (valid) {
            double *o = a.out + gout * (NAB * NCD);
#pragma unroll
            for (int e = 0; e < NAB * NCD; ++e) o[e] = (double)V[e];
        }
        return;
    } else {
        const int n = a.nao;
        for (int s = 0; s < a.nset; ++s) {
            const double *D = a.D + s * a.mstride;
            double *Jm = a.J + s * a.mstride;
            double *Km = a.K + s * a.mstride;
            if (a.do_j) {
                double dij[NAB], dkl[NCD];
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) dij[i * NJ + j] = D[(B.aoi + i) * n + B.aoj + j];
#pragma unroll
                for (int k = 0; k < NK; ++k)
#pragma unroll
                    for (int l = 0; l < NL; ++l) dkl[k * NL + l] = D[(Kt.aoi + k) * n + Kt.aoj + l];
                const double w2 = valid ? 2.0 * wq : 0.0;
                if constexpr (BRA_UNIFORM) {
                    // J_IJ: reduce over the wave's kets
                    // lane e holds the reduced elements e, e + 64, ...
                    constexpr int NM = (NAB + 63) / 64;
                    double mine[NM];
#pragma unroll
                    for (int m = 0; m < NM; ++m) mine[m] = 0.0;
#pragma unroll
                    for (int ab2 = 0; ab2 < NAB; ++ab2) {
                        double s2 = 0.0;
#pragma unroll
                        for (int cd2 = 0; cd2 < NCD; ++cd2) s2 += (double)V[ab2 * NCD + cd2] * dkl[cd2];
                        s2 = wave_sum(s2 * w2);
                        if (lane == ab2 % 64) mine[ab2 / 64] = s2;
                    }
#pragma unroll
                    for (int m = 0; m < NM; ++m) {
                        const int e = lane + 64 * m;
                        if (e < NAB) acc_add(a, &Jm[(B.aoi + e / NJ) * n + B.aoj + e % NJ], mine[m]);
                    }
                } else if (valid) {
#pragma unroll
                    for (int ab2 = 0; ab2 < NAB; ++ab2) {
                        double s2 = 0.0;
#pragma unroll
                        for (int cd2 = 0; cd2 < NCD; ++cd2) s2 += (double)V[ab2 * NCD + cd2] * dkl[cd2];
                        acc_add(a, &Jm[(B.aoi + ab2 / NJ) * n + B.aoj + ab2 % NJ], w2 * s2);
                    }
                }
                if (valid) {
                    // J'_KL into the pair-ordered buffer (consecutive kets,
                    // consecutive addresses)
                    double *jq = a.jp + s * a.jpstride + Kt.jp_off;
#pragma unroll
                    for (int cd2 = 0; cd2 < NCD; ++cd2) {
                        double s2 = 0.0;
#pragma unroll
                        for (int ab2 = 0; ab2 < NAB; ++ab2) s2 += (double)V[ab2 * NCD + cd2] * dij[ab2];
                        acc_add(a, &jq[(int64_t)cd2 * Kt.pp_stride], w2 * s2);
                    }
                }
            }
            if (a.do_k && valid) {
                double djl[NJ * NL], djk[NJ * NK], dil[NI * NL], dik[NI * NK];
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
#pragma unroll
                    for (int l = 0; l < NL; ++l) djl[j * NL + l] = D[(B.aoj + j) * n + Kt.aoj + l];
#pragma unroll
                    for (int k = 0; k < NK; ++k) djk[j * NK + k] = D[(B.aoj + j) * n + Kt.aoi + k];
                }
#pragma unroll
                for (int i = 0; i < NI; ++i) {
#pragma unroll
                    for (int l = 0; l < NL; ++l) dil[i * NL + l] = D[(B.aoi + i) * n + Kt.aoj + l];
#pragma unroll
                    for (int k = 0; k < NK; ++k) dik[i * NK + k] = D[(B.aoi + i) * n + Kt.aoi + k];
                }
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int k = 0; k < NK; ++k) {
                        double s2 = 0.0;
#pragma unroll
                        for (int j = 0; j < NJ; ++j)
#pragma unroll
                            for (int l = 0; l < NL; ++l) s2 += (double)V[((i * NJ + j) * NK + k) * NL + l] * djl[j * NL + l];
                        acc_add(a, &Km[(B.aoi + i) * n + Kt.aoi + k], wq * s2);
                    }
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        double s2 = 0.0;
#pragma unroll
                        for (int j = 0; j < NJ; ++j)
#pragma unroll
                            for (int k = 0; k < NK; ++k) s2 += (double)V[((i * NJ + j) * NK + k) * NL + l] * djk[j * NK + k];
                        acc_add(a, &Km[(B.aoi + i) * n + Kt.aoj + l], wq * s2);
                    }
#pragma unroll
                for (int j = 0; j < NJ; ++j)
#pragma unroll
                    for (int k = 0; k < NK; ++k) {
                        double s2 = 0.0;
#pragma unroll
                        for (int i = 0; i < NI; ++i)
#pragma unroll
                            for (int l = 0; l < NL; ++l) s2 += (double)V[((i * NJ + j) * NK + k) * NL + l] * dil[i * NL + l];
                        acc_add(a, &Km[(B.aoj + j) * n + Kt.aoi + k], wq * s2);
                    }
#pragma unroll
                for (int j = 0; j < NJ; ++j)
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        double s2 = 0.0;
#pragma unroll
                        for (int i = 0; i < NI; ++i)
#pragma unroll
                            for (int k = 0; k < NK; ++k) s2 += (double)V[((i * NJ + j) * NK + k) * NL + l] * dik[i * NK + k];
                        acc_add(a, &Km[(B.aoj + j) * n + Kt.aoj + l], wq * s2);
                    }
            }
        }
    }
}

// One tile (64 kets of one bra) for one wave.
template <int LI, int LJ, int LK, int LL, typename R>
__device__ __forceinline__ void k1_tile(const JkArgs &a, int wave) {
    const int lane = lane_index();
    {
        const int i = tile_bra(a.tile_off, a.nbra, wave);
        const int j0 = (wave - a.tile_off[i]) * 64, j = j0 + lane;
        const int cnt = a.bra_cnt[i];
        bool valid = j < cnt;
        const int bra = a.bra_list[i];
        const PairRec &B = a.pairs[bra];
        if (!prefix_selectable(a, B.q, a.pairs[a.ket_list[j0]].q)) return;
        const int ket = a.ket_list[valid ? j : cnt - 1];
        const PairRec &Kt = a.pairs[ket];
        const double wq = pair_weight(bra, ket, B, Kt);
        screen_quartet(a, B, Kt, valid);
        const int n = count_selected(valid);
        if (n == 0) return;
        add_count(a, n);
        k1_body<LI, LJ, LK, LL, R, MODE_JK>(a, bra, ket, valid, wq, 0);
    }
}

// Tiles: one wave per tile of 64 kets of one bra.
template <int LI, int LJ, int LK, int LL, typename R, int MODE>
__global__ void __launch_bounds__(256) jk_k1(const JkArgs a) {
    if constexpr (MODE == MODE_JK) {
        const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
        if (wave >= a.ntiles) return;
        k1_tile<LI, LJ, LK, LL, R>(a, wave);
    } else {
        const int g = blockIdx.x * 256 + threadIdx.x;
        const bool valid = g < a.nq;
        const int gg = valid ? g : a.nq - 1;
        k1_body<LI, LJ, LK, LL, R, MODE_EXPORT>(a, a.q_bra[gg], a.q_ket[gg], valid, 1.0, g);
    }
}

struct BatchDesc {
    JkArgs a;
    int32_t tile_base;
    int32_t pad[3];
};

// The argument block of descriptor m.  The descriptors are written before
// the launch and only read by the kernels, so they are read through the
// constant address space: the compiler may then load a field where it is
// used (and load it again later) instead of holding the whole block in
// registers, which made the batched family-1 row kernels spill.
__device__ __forceinline__ const JkArgs &desc_args(const BatchDesc *descs, int m) {
    using CDesc = const __attribute__((address_space(4))) BatchDesc;
    return *(const JkArgs *)&((CDesc *)descs)[m].a;
}

__device__ __forceinline__ int batch_desc(const BatchDesc *__restrict__ d, int n, int g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile_base <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Row mode: one workgroup of NT lanes walks a chunk of one bra's ket prefix
// (a row task: list position, first and end ket).  K'_IK, K'_IL (row block
// of shell I) and K'_JK, K'_JL (row block of J) accumulate in LDS over the
// compressed ket-type columns, J'_IJ in LDS, and only J'_KL leaves per
// quartet (atomics into the pair-ordered buffer).  Dynamic LDS layout: the bra's npb primitive pair
// records, then per density [NI rows | NJ rows] x ncols and NAB for J'_IJ.
// NT = 256 for long bras, 64 for short ones;
// BATCH: the task indexes the row tasks of many descriptors (molecules).
template <int LI, int LJ, int LK, int LL, typename R, int NT>
__device__ __forceinline__ void k1_row_task(const JkArgs &a, int task) {
    using C = Cls<LI, LJ, LK, LL>;
    constexpr int NI = C::NI, NJ = C::NJ, NK = C::NK, NL = C::NL, NAB = C::NAB, NCD = C::NCD;
    extern __shared__ double rowmem[];
    const int tid = threadIdx.x, lane = lane_index();
    const int i = a.row_pos[3 * task];
    const int jbeg = a.row_pos[3 * task + 1], cnt = a.row_pos[3 * task + 2];
    const int bra = a.bra_list[i];
    const int ncols = a.ncolK + (a.seg_same ? 0 : a.ncolL);
    const int segL = a.seg_same ? 0 : a.ncolK;
    const int per_set = (NI + NJ) * ncols + NAB;
    const PairRec B = a.pairs[bra];
    // a task none of whose quartets can be selected ends here (uniform in the workgroup)
    if (!prefix_selectable(a, B.q, a.pairs[a.ket_list[jbeg]].q)) return;
    // the bra's primitive pair records, then the rows
    PrimPair *sbra = reinterpret_cast<PrimPair *>(rowmem);
    double *rows = rowmem + (size_t)a.npb * (sizeof(PrimPair) / sizeof(double));
    // staged D rows of the bra (a.dstage): [nset][NI + NJ][ncols], column c
    // holding the AO of the K row's column c
    // (compiled in for the small bras only, where it can fit the LDS budget)
    constexpr bool DST = k1_dstage_class(LI, LJ);
    const bool dstage = DST && a.dstage;
    const int dper = (NI + NJ) * ncols;
    double *drows = rows + (size_t)per_set * a.nset;
    const int n = a.nao;
    for (int t = tid; t < a.npb; t += NT) sbra[t] = a.pp[B.pp_off + t * B.pp_stride];
    for (int t = tid; t < per_set * a.nset; t += NT) rows[t] = 0.0;
    if (dstage) {
        for (int t = tid; t < dper * a.nset; t += NT) {
            const int s = t / dper, e = t - s * dper;
            const int r = e / ncols, c = e - r * ncols;
            const int row = r < NI ? B.aoi + r : B.aoj + (r - NI);
            const int col = c < a.ncolK ? a.aoc[a.tshK[c / NK]] + c % NK
                                        : a.aoc[a.tshL[(c - a.ncolK) / NL]] + (c - a.ncolK) % NL;
            drows[t] = a.D[s * a.mstride + (int64_t)row * n + col];
        }
    }
    __syncthreads();
    int evaluated = 0;  // quartets this wave evaluated (wave-uniform)
    for (int j0 = jbeg; j0 < cnt; j0 += NT) {
        if (!prefix_selectable(a, B.q, a.pairs[a.ket_list[j0]].q)) break;  // uniform in the workgroup
        const int j = j0 + tid;
        bool valid = j < cnt;
        const int ket = a.ket_list[valid ? j : cnt - 1];
        const PairRec Kt = a.pairs[ket];
        const double wq = pair_weight(bra, ket, B, Kt);
        screen_quartet(a, B, Kt, valid);
        // (no workgroup barrier inside this loop: a wave may skip a pass)
        const int nv = count_selected(valid);
        if (nv == 0) continue;
        evaluated += nv;
        R V[C::NC];
        k1_compute<LI, LJ, LK, LL, R>(a, B, Kt, [&](int ib) { return sbra[ib]; }, a.npb, a.npk, V);
        const int cK = a.tpos[Kt.ish] * NK, cL = segL + a.tpos[Kt.jsh] * NL;
        for (int s = 0; s < a.nset; ++s) {
            const double *D = a.D + s * a.mstride;
            double *rm = rows + s * per_set;
            double *rI = rm, *rJ = rm + NI * ncols, *jij = rm + (NI + NJ) * ncols;
            if (a.do_j) {
                double dij[NAB], dkl[NCD];
#pragma unroll
                for (int i2 = 0; i2 < NI; ++i2)
#pragma unroll
                    for (int j2 = 0; j2 < NJ; ++j2) dij[i2 * NJ + j2] = D[(B.aoi + i2) * n + B.aoj + j2];
#pragma unroll
                for (int k = 0; k < NK; ++k)
#pragma unroll
                    for (int l = 0; l < NL; ++l) dkl[k * NL + l] = D[(Kt.aoi + k) * n + Kt.aoj + l];
                const double w2 = valid ? 2.0 * wq : 0.0;
                constexpr int NM = (NAB + 63) / 64;
                double mine[NM];
#pragma unroll
                for (int m = 0; m < NM; ++m) mine[m] = 0.0;
#pragma unroll
                for (int ab2 = 0; ab2 < NAB; ++ab2) {
                    double s2 = 0.0;
#pragma unroll
                    for (int cd2 = 0; cd2 < NCD; ++cd2) s2 += (double)V[ab2 * NCD + cd2] * dkl[cd2];
                    s2 = wave_sum(s2 * w2);
                    if (lane == ab2 % 64) mine[ab2 / 64] = s2;
                }
#pragma unroll
                for (int m = 0; m < NM; ++m)
                    if (lane + 64 * m < NAB) atomicAdd(&jij[lane + 64 * m], mine[m]);
                if (valid) {
                    double *jq = a.jp + s * a.jpstride + Kt.jp_off;
#pragma unroll
                    for (int cd2 = 0; cd2 < NCD; ++cd2) {
                        double s2 = 0.0;
#pragma unroll
                        for (int ab2 = 0; ab2 < NAB; ++ab2) s2 += (double)V[ab2 * NCD + cd2] * dij[ab2];
                        atomic_add_f64(&jq[(int64_t)cd2 * Kt.pp_stride], w2 * s2);
                    }
                }
            }
            if (a.do_k && valid) {
                double djl[NJ * NL], djk[NJ * NK], dil[NI * NL], dik[NI * NK];
                if (dstage) {
                    const double *dr = drows + s * dper;
#pragma unroll
                    for (int j2 = 0; j2 < NJ; ++j2) {
#pragma unroll
                        for (int l = 0; l < NL; ++l) djl[j2 * NL + l] = dr[(NI + j2) * ncols + cL + l];
#pragma unroll
                        for (int k = 0; k < NK; ++k) djk[j2 * NK + k] = dr[(NI + j2) * ncols + cK + k];
                    }
#pragma unroll
                    for (int i2 = 0; i2 < NI; ++i2) {
#pragma unroll
                        for (int l = 0; l < NL; ++l) dil[i2 * NL + l] = dr[i2 * ncols + cL + l];
#pragma unroll
                        for (int k = 0; k < NK; ++k) dik[i2 * NK + k] = dr[i2 * ncols + cK + k];
                    }
                } else {
#pragma unroll
                    for (int j2 = 0; j2 < NJ; ++j2) {
#pragma unroll
                        for (int l = 0; l < NL; ++l) djl[j2 * NL + l] = D[(B.aoj + j2) * n + Kt.aoj + l];
#pragma unroll
                        for (int k = 0; k < NK; ++k) djk[j2 * NK + k] = D[(B.aoj + j2) * n + Kt.aoi + k];
                    }
#pragma unroll
                    for (int i2 = 0; i2 < NI; ++i2) {
#pragma unroll
                        for (int l = 0; l < NL; ++l) dil[i2 * NL + l] = D[(B.aoi + i2) * n + Kt.aoj + l];
#pragma unroll
                        for (int k = 0; k < NK; ++k) dik[i2 * NK + k] = D[(B.aoi + i2) * n + Kt.aoi + k];
                    }
                }
#pragma unroll
                for (int i2 = 0; i2 < NI; ++i2)
#pragma unroll
                    for (int k = 0; k < NK; ++k) {
                        double s2 = 0.0;
#pragma unroll
                        for (int j2 = 0; j2 < NJ; ++j2)
#pragma unroll
                            for (int l = 0; l < NL; ++l)
                                s2 += (double)V[((i2 * NJ + j2) * NK + k) * NL + l] * djl[j2 * NL + l];
                        atomicAdd(&rI[i2 * ncols + cK + k], wq * s2);
                    }
#pragma unroll
                for (int i2 = 0; i2 < NI; ++i2)
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        double s2 = 0.0;
#pragma unroll
                        for (int j2 = 0; j2 < NJ; ++j2)
#pragma unroll
                            for (int k = 0; k < NK; ++k)
                                s2 += (double)V[((i2 * NJ + j2) * NK + k) * NL + l] * djk[j2 * NK + k];
                        atomicAdd(&rI[i2 * ncols + cL + l], wq * s2);
                    }
#pragma unroll
                for (int j2 = 0; j2 < NJ; ++j2)
#pragma unroll
                    for (int k = 0; k < NK; ++k) {
                        double s2 = 0.0;
#pragma unroll
                        for (int i2 = 0; i2 < NI; ++i2)
#pragma unroll
                            for (int l = 0; l < NL; ++l)
                                s2 += (double)V[((i2 * NJ + j2) * NK + k) * NL + l] * dil[i2 * NL + l];
                        atomicAdd(&rJ[j2 * ncols + cK + k], wq * s2);
                    }
#pragma unroll
                for (int j2 = 0; j2 < NJ; ++j2)
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        double s2 = 0.0;
#pragma unroll
                        for (int i2 = 0; i2 < NI; ++i2)
#pragma unroll
                            for (int k = 0; k < NK; ++k)
                                s2 += (double)V[((i2 * NJ + j2) * NK + k) * NL + l] * dik[i2 * NK + k];
                        atomicAdd(&rJ[j2 * ncols + cL + l], wq * s2);
                    }
            }
        }
    }
    add_count(a, evaluated);
    __syncthreads();
    // flush nonzero entries to the global J', K'
    for (int s = 0; s < a.nset; ++s) {
        const double *rm = rows + s * per_set;
        double *Jm = a.J + s * a.mstride;
        double *Km = a.K + s * a.mstride;
        for (int t = tid; t < per_set; t += NT) {
            const double v = rm[t];
            if (v == 0.0) continue;
            if (t >= (NI + NJ) * ncols) {
                const int e = t - (NI + NJ) * ncols;
                atomic_add_f64(&Jm[(B.aoi + e / NJ) * n + B.aoj + e % NJ], v);
                continue;
            }
            const int r = t / ncols, c = t % ncols;
            const int row = r < NI ? B.aoi + r : B.aoj + (r - NI);
            int col;
            if (c < a.ncolK) col = a.aoc[a.tshK[c / NK]] + c % NK;
            else col = a.aoc[a.tshL[(c - a.ncolK) / NL]] + (c - a.ncolK) % NL;
            atomic_add_f64(&Km[row * n + col], v);
        }
    }
}

// Waves per SIMD the compiler is held to for a family-1 row kernel: five
// for the FP64 (ps|ss) class (96 VGPRs; left to itself it takes 101, four
// waves), none otherwise.
constexpr int k1_row_waves(int li, int lj, int lk, int ll, int rsize) {
    return (li + lj + lk + ll == 1 && rsize == 8) ? 5 : 1;
}
template <int LI, int LJ, int LK, int LL, typename R, int NT, bool BATCH>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(k1_row_waves(LI, LJ, LK, LL, sizeof(R)))))
jk_k1_row(const JkArgs a, const BatchDesc *__restrict__ descs, int ndesc) {
    if constexpr (BATCH) {
        const int g = blockIdx.x;
        const int m = __builtin_amdgcn_readfirstlane(batch_desc(descs, ndesc, g));
        k1_row_task<LI, LJ, LK, LL, R, NT>(desc_args(descs, m), g - descs[m].tile_base);
    } else {
        k1_row_task<LI, LJ, LK, LL, R, NT>(a, blockIdx.x);
    }
}

// ===========================================================================
// Family 2: a lane group per quartet.  Lane slot (a, c) owns the elements
// (a b | c d) for all b in the current pass's chunk and all d.  Per
// primitive quartet, lanes first evaluate the roots and weights (one lane
// per root) into LDS, then build the 2-D tables I_x, I_y, I_z of every root
// into LDS (one task = one root and direction), then every slot accumulates
// its elements from LDS.  Digestion: per slot partial sums, reduced across
// the group in LDS, then one FP64 global atomic per block element.
// ===========================================================================
template <int LI, int LJ, int LK, int LL>
struct K2Cfg {
    using C = Cls<LI, LJ, LK, LL>;
    static constexpr int NSLOT = C::NI * C::NK;
    static constexpr int QW = k2_qw(LI, LJ, LK, LL);
    static constexpr int LPQ = QW > 1 ? NSLOT : 64;          // lanes per quartet
    static constexpr int SPL = (NSLOT + LPQ - 1) / LPQ;       // slots per lane
    // b-chunk per pass: keep SPL * CB * NL accumulators <= 48
    static constexpr int cb_() {
        int cb = C::NJ;
        while (cb > 1 && SPL * cb * C::NL > 48) --cb;
        return cb;
    }
    static constexpr int CB = cb_();
    static constexpr int NPASS = (C::NJ + CB - 1) / CB;
    // roots whose tables are held at once: all of them where the wave's
    // tables fit 56 KB (in FP64), otherwise blocks of RB roots within 48 KB
    // one after another.  Blocks cost a table build per block and b-chunk
    // pass (the tables of one block do not outlive the pass), which the
    // classes whose tables take 49-53 KB ((gf|ff), (gf|gd), (gg|fd)) lose
    // more to than to the lower occupancy of the larger LDS block; above
    // that the occupancy loss dominates.
    static constexpr int TAB_ALL = 56 * 1024, TAB_BLK = 48 * 1024;
    static constexpr int RB = (QW * C::NR * 3 * C::S * 8 <= TAB_ALL) ? C::NR
                              : (TAB_BLK / (QW * 3 * C::S * 8) > 0 ? TAB_BLK / (QW * 3 * C::S * 8) : 1);
    static constexpr int NRB = (C::NR + RB - 1) / RB;
    // roots of a block unrolled in the accumulation: all of them while a
    // root's products are few; above that the unrolled block keeps more
    // table values in flight than the register file holds (the kernels
    // spilled up to 2.5 KB per lane), so the roots then run as a loop
    static constexpr int RUNROLL = SPL * CB * C::NL * RB > 96 ? 1 : RB;
    // primitive quartets whose tables are built at once: enough that every
    // lane of a quartet's group has a (primitive, root, direction) task,
    // within 24 KB of tables per wave (in FP64); one where the roots come in
    // blocks
    static constexpr int pb_() {
        if (NRB > 1) return 1;
        int pb = LPQ / (3 * C::NR);
        const int cap = (24 * 1024) / (QW * C::NR * 3 * C::S * 8);
        if (pb > cap) pb = cap;
        return pb < 1 ? 1 : pb;
    }
    static constexpr int PB = pb_();
    // one (primitive, root, direction) table is S entries, stored SP apart:
    // an odd stride, so the table-building lanes of a wave (one table each)
    // write to different LDS banks
    static constexpr int SP = C::S % 2 == 0 ? C::S + 1 : C::S;
    static constexpr int TAB = PB * RB * 3 * SP;              // 2-D table entries per quartet
    // LDS digestion blocks: jij, jkl, kik, kil, kjk, kjl
    static constexpr int O_JIJ = 0;
    static constexpr int O_JKL = O_JIJ + C::NI * C::NJ;
    static constexpr int O_KIK = O_JKL + C::NK * C::NL;
    static constexpr int O_KIL = O_KIK + C::NI * C::NK;
    static constexpr int O_KJK = O_KIL + C::NI * C::NL;
    static constexpr int O_KJL = O_KJK + C::NJ * C::NK;
    static constexpr int DIG = O_KJL + C::NJ * C::NL;
    // per wave: the QW digestion blocks, then every lane's partial K_JL
    // sums of a pass ([lane][b in pass][d]), reduced over the slots without
    // atomics
    static constexpr int PARTW = 64 * CB * C::NL;
    static constexpr int DIGW = QW * DIG + PARTW;
    // table index [ax][cx][bx][dx]
    static __device__ __forceinline__ constexpr int tix(int ax, int bx, int cx, int dx) {
        return ((ax * (LK + 1) + cx) * (LJ + 1) + bx) * (LL + 1) + dx;
    }
};

// One wave handles QW quartets with its own tables and digestion blocks;
// the tables of PB primitive quartets are built at once (every lane of a
// quartet's group takes a (primitive, root, direction) task) and then
// consumed one after another;
// all synchronisation inside is per wave, so the waves of a workgroup are
// independent.  ROW: the four K blocks and J_IJ go to the
// workgroup's shared K rows of the (uniform) bra instead (row mode), only
// J_KL is flushed per quartet.
template <int LI, int LJ, int LK, int LL, typename R, int MODE, bool ROW = false>
__device__ __forceinline__ void k2_body(const JkArgs &a, R *tabs, double *dig, int bra, int ket, bool valid, double wq,
                                        int64_t gq, double *rows = nullptr, int ncols = 0, int segL = 0) {
    using C = Cls<LI, LJ, LK, LL>;
    using F = K2Cfg<LI, LJ, LK, LL>;
    constexpr int NI = C::NI, NJ = C::NJ, NK = C::NK, NL = C::NL, NR = C::NR, S = F::SP;
    constexpr int QW = F::QW, LPQ = F::LPQ, SPL = F::SPL, CB = F::CB, NPASS = F::NPASS, PB = F::PB;
    const int lane = lane_index();
    const int q = QW > 1 ? lane / LPQ : 0;
    const int sl = QW > 1 ? lane % LPQ : lane;
    const bool lane_used = q < QW;
    const int qq = lane_used ? q : 0;
    const PairRec B = a.pairs[bra];
    const PairRec Kt = a.pairs[ket];
    const int npb = MODE == MODE_JK ? a.npb : B.npp;
    const int npk = MODE == MODE_JK ? a.npk : Kt.npp;
    const int npq = npb * npk;
    int npq_max = npq;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) npq_max = max(npq_max, __shfl_xor(npq_max, off, 64));

    R *tq = tabs + qq * F::TAB;
    double *dq = dig + qq * F::DIG;

    int sa[SPL], sc[SPL];
    bool sv[SPL];
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
        const int slot = sl + k * LPQ;
        sv[k] = lane_used && slot < F::NSLOT;
        const int s2 = sv[k] ? slot : 0;
        sa[k] = s2 / NK;
        sc[k] = s2 % NK;
    }
    int base[SPL][3];
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
        int ae[3] = {0, 0, 0}, ce[3] = {0, 0, 0};
#pragma unroll
        for (int t = 0; t < NI; ++t)
            if (t == sa[k]) { ae[0] = cart_comp(LI, t, 0); ae[1] = cart_comp(LI, t, 1); ae[2] = cart_comp(LI, t, 2); }
#pragma unroll
        for (int t = 0; t < NK; ++t)
            if (t == sc[k]) { ce[0] = cart_comp(LK, t, 0); ce[1] = cart_comp(LK, t, 1); ce[2] = cart_comp(LK, t, 2); }
#pragma unroll
        for (int x = 0; x < 3; ++x) base[k][x] = x * S + F::tix(ae[x], 0, ce[x], 0);
    }
    const R ab[3] = {(R)B.ab[0], (R)B.ab[1], (R)B.ab[2]};
    const R cd[3] = {(R)Kt.ab[0], (R)Kt.ab[1], (R)Kt.ab[2]};

#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        R acc[SPL][CB][NL];
#pragma unroll
        for (int k = 0; k < SPL; ++k)
#pragma unroll
            for (int bb = 0; bb < CB; ++bb)
#pragma unroll
                for (int d = 0; d < NL; ++d) acc[k][bb][d] = (R)0;

        // every primitive quartet once per operator variant, PB of them per
        // table build
        const int vb = variant_begin(a.omega), nv = variant_end(a.omega) - vb;
        const int nit = npq_max * nv;
        for (int it0 = 0; it0 < nit; it0 += PB) {
            // with a single table set per quartet the tables of pass 0 are
            // reused by the later passes
            const bool build = pass == 0 || nit > PB || F::NRB > 1;
#pragma unroll
            for (int rb = 0; rb < F::NRB; ++rb) {
            constexpr int RB = F::RB;
            const int r0 = rb * RB, nrb = NR - r0 < RB ? NR - r0 : RB;  // roots of this block
            if (build) {
                wave_sync();
                // one task per (primitive quartet of the batch, root, direction)
                for (int t = sl; t < PB * 3 * nrb && lane_used; t += LPQ) {
                    const int p = t / (3 * nrb), t2 = t - p * (3 * nrb);
                    const int it = it0 + p;
                    const int ipq = it / nv, var = vb + it % nv;
                    const bool has = it < nit && ipq < npq;
                    const int ib = has ? ipq % npb : 0, ik = has ? ipq / npb : 0;
                    const PrimPair pb = a.pp[B.pp_off + ib * B.pp_stride];
                    const PrimPair pk = a.pp[Kt.pp_off + ik * Kt.pp_stride];
                    const PQuart<R> g = prim_quartet<R>(pb, pk);
                    const int rl = t2 / 3, r = r0 + rl, x = t2 % 3;
                    R u, w;
                    rys_root1_op<NR, R>(g.T, g.rho, a.omega, var, r, a.tab, u, w);
                    const R b00 = (R)0.5 * u * g.rpq;
                    const R b10 = g.hb * ((R)1 - g.fq * u);
                    const R b01 = g.hk * ((R)1 - g.fp * u);
                    // the direction's operands by value selects (an indexed
                    // read makes the compiler keep a scratch copy of them)
                    const R pqx = sel3(x, g.PQ[0], g.PQ[1], g.PQ[2]);
                    const R pax = sel3(x, g.PA[0], g.PA[1], g.PA[2]);
                    const R qcx = sel3(x, g.QC[0], g.QC[1], g.QC[2]);
                    const R abx = sel3(x, ab[0], ab[1], ab[2]);
                    const R cdx = sel3(x, cd[0], cd[1], cd[2]);
                    const R c00 = pax - g.fq * u * pqx;
                    const R c00p = qcx + g.fp * u * pqx;
                    const R sc2 = x == 2 ? (has ? w * g.pref : (R)0) : (R)1;
                    R *dst = tq + ((p * RB + rl) * 3 + x) * S;
                    rys2d<LI, LJ, LK, LL, R>(c00, c00p, b00, b10, b01, abx, cdx, sc2,
                                             [&](int ia, int ib2, int ic, int id, R v) { dst[F::tix(ia, ib2, ic, id)] = v; });
                }
                wave_sync();
            }
            for (int p = 0; p < PB; ++p) {
            if (it0 + p >= nit) break;  // uniform in the wave
#pragma unroll F::RUNROLL
            for (int rl = 0; rl < RB; ++rl) {
                if (r0 + rl >= NR) continue;
                const R *tr = tq + (p * RB + rl) * 3 * S;
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
#pragma unroll
                    for (int bb = 0; bb < CB; ++bb) {
                        const int b = pass * CB + bb;
                        if (b >= NJ) continue;
#pragma unroll
                        for (int d = 0; d < NL; ++d) {
                            const int ox = F::tix(0, cart_comp(LJ, b, 0), 0, cart_comp(LL, d, 0));
                            const int oy = F::tix(0, cart_comp(LJ, b, 1), 0, cart_comp(LL, d, 1));
                            const int oz = F::tix(0, cart_comp(LJ, b, 2), 0, cart_comp(LL, d, 2));
                            acc[k][bb][d] += tr[base[k][0] + ox] * tr[base[k][1] + oy] * tr[base[k][2] + oz];
                        }
                    }
                }
            }
            }  // primitive quartet of the batch
            }  // root block
        }

        if constexpr (MODE == MODE_EXPORT) {
#pragma unroll
            for (int k = 0; k < SPL; ++k) {
                if (!(valid && sv[k])) continue;
                double *o = a.out + gq * C::NC;
#pragma unroll
                for (int bb = 0; bb < CB; ++bb) {
                    const int b = pass * CB + bb;
                    if (b >= NJ) continue;
#pragma unroll
                    for (int d = 0; d < NL; ++d) o[((sa[k] * NJ + b) * NK + sc[k]) * NL + d] = (double)acc[k][bb][d];
                }
            }
        } else {
            const int n = a.nao;
            // row mode: compressed K-row columns of this quartet's ket shells
            const int cK = ROW ? a.tpos[Kt.ish] * NK : 0, cL = ROW ? segL + a.tpos[Kt.jsh] * NL : 0;
            const int per_set = (NI + NJ) * ncols + NI * NJ;
            for (int s = 0; s < a.nset; ++s) {
                const double *D = a.D + s * a.mstride;
                double *rI = rows + s * per_set, *rJ = rI + NI * ncols, *rjij = rI + (NI + NJ) * ncols;
                wave_sync();
                for (int t = lane; t < QW * F::DIG; t += 64) dig[t] = 0.0;
                wave_sync();
                double kjlp[CB][NL];
#pragma unroll
                for (int bb = 0; bb < CB; ++bb)
#pragma unroll
                    for (int d = 0; d < NL; ++d) kjlp[bb][d] = 0.0;
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
                    if (!(valid && sv[k])) continue;
                    const int ia = sa[k], ic = sc[k];
                    const int ga = B.aoi + ia, gc = Kt.aoi + ic;
                    double dkl[NL], dil[NL];
#pragma unroll
                    for (int d = 0; d < NL; ++d) {
                        dkl[d] = D[gc * n + Kt.aoj + d];
                        dil[d] = D[ga * n + Kt.aoj + d];
                    }
                    const double dik = D[ga * n + gc];
                    double kik = 0.0, jkl[NL], kil[NL];
#pragma unroll
                    for (int d = 0; d < NL; ++d) { jkl[d] = 0.0; kil[d] = 0.0; }
#pragma unroll
                    for (int bb = 0; bb < CB; ++bb) {
                        const int b = pass * CB + bb;
                        if (b >= NJ) continue;
                        const int gb = B.aoj + b;
                        const double dij = D[ga * n + gb];
                        const double djk = D[gb * n + gc];
                        double jij = 0.0, kjk = 0.0;
#pragma unroll
                        for (int d = 0; d < NL; ++d) {
                            const double v = (double)acc[k][bb][d];
                            const double djl = D[gb * n + Kt.aoj + d];
                            jij += v * dkl[d];
                            jkl[d] += v * dij;
                            kik += v * djl;
                            kil[d] += v * djk;
                            kjk += v * dil[d];
                            kjlp[bb][d] += v * dik;
                        }
                        if (a.do_j) atomicAdd(ROW ? &rjij[ia * NJ + b] : &dq[F::O_JIJ + ia * NJ + b], 2.0 * wq * jij);
                        if (a.do_k) atomicAdd(ROW ? &rJ[b * ncols + cK + ic] : &dq[F::O_KJK + b * NK + ic], wq * kjk);
                    }
#pragma unroll
                    for (int d = 0; d < NL; ++d) {
                        if (a.do_j) atomicAdd(&dq[F::O_JKL + ic * NL + d], 2.0 * wq * jkl[d]);
                        if (a.do_k) atomicAdd(ROW ? &rI[ia * ncols + cL + d] : &dq[F::O_KIL + ia * NL + d], wq * kil[d]);
                    }
                    if (a.do_k) atomicAdd(ROW ? &rI[ia * ncols + cK + ic] : &dq[F::O_KIK + ia * NK + ic], wq * kik);
                }
                // K_JL of each quartet: the sum of its lanes' partials (every
                // slot of the quartet adds to the same elements), reduced
                // through LDS without atomics; in row mode one LDS atomic per
                // element then adds it to the bra's K row, at the quartet's
                // ket column (kept in the quartet's unused K_JL digestion slot)
                if (a.do_k) {
                    double *part = dig + QW * F::DIG;
                    if constexpr (ROW) {
                        if (lane_used && sl == 0) dq[F::O_KJL] = (double)cL;
                    }
#pragma unroll
                    for (int bb = 0; bb < CB; ++bb)
#pragma unroll
                        for (int d = 0; d < NL; ++d) part[lane * (CB * NL) + bb * NL + d] = wq * kjlp[bb][d];
                    wave_sync();
                    for (int t = lane; t < QW * CB * NL; t += 64) {
                        const int q2 = t / (CB * NL), bd = t % (CB * NL);
                        const int b = pass * CB + bd / NL;
                        if (b >= NJ) continue;
                        double sum = 0.0;
                        for (int l2 = 0; l2 < LPQ; ++l2) sum += part[(q2 * LPQ + l2) * (CB * NL) + bd];
                        if constexpr (ROW) {
                            if (sum != 0.0) atomicAdd(&rJ[b * ncols + (int)dig[q2 * F::DIG + F::O_KJL] + bd % NL], sum);
                        } else {
                            dig[q2 * F::DIG + F::O_KJL + b * NL + bd % NL] = sum;
                        }
                    }
                }
                wave_sync();
                if (lane_used && valid) {
                    double *Jm = a.J + s * a.mstride;
                    double *Km = a.K + s * a.mstride;
                    const int t0 = ROW ? F::O_JKL : 0, t1 = ROW ? F::O_KIK : F::DIG;
                    for (int t = t0 + sl; t < t1; t += LPQ) {
                        const double v = dq[t];
                        if (v == 0.0) continue;
                        int row, col;
                        double *M;
                        if (t < F::O_JKL) { row = B.aoi + t / NJ; col = B.aoj + t % NJ; M = Jm; }
                        else if (t < F::O_KIK) { const int e = t - F::O_JKL; row = Kt.aoi + e / NL; col = Kt.aoj + e % NL; M = Jm; }
                        else if (t < F::O_KIL) { const int e = t - F::O_KIK; row = B.aoi + e / NK; col = Kt.aoi + e % NK; M = Km; }
                        else if (t < F::O_KJK) { const int e = t - F::O_KIL; row = B.aoi + e / NL; col = Kt.aoj + e % NL; M = Km; }
                        else if (t < F::O_KJL) { const int e = t - F::O_KJK; row = B.aoj + e / NK; col = Kt.aoi + e % NK; M = Km; }
                        else { const int e = t - F::O_KJL; row = B.aoj + e / NL; col = Kt.aoj + e % NL; M = Km; }
                        acc_add(a, &M[row * n + col], v);
                    }
                }
            }
        }
    }
}

// One tile (QW kets of one bra) for the one-wave workgroup, expanded in
// place in each kernel.  As a helper function taking the LDS arrays as
// pointers, the compiler kept the large FP64 classes' accumulators in
// scratch (four times the private memory of the in-place form) and the
// (ff|ff) kernel returned wrong values.
#define JK_K2_TILE(a, wave)                                                     \
    do {                                                                        \
        const int i_ = tile_bra((a).tile_off, (a).nbra, (wave));                \
        const int j0_ = ((wave) - (a).tile_off[i_]) * QW;                       \
        const int j_ = j0_ + qq;                                                \
        const int cnt_ = (a).bra_cnt[i_];                                       \
        bool valid_ = lane_used && j_ < cnt_;                                   \
        const int bra_ = (a).bra_list[i_];                                      \
        if (!prefix_selectable((a), (a).pairs[bra_].q, (a).pairs[(a).ket_list[j0_]].q)) break; \
        const int ket_ = (a).ket_list[j_ < cnt_ ? j_ : cnt_ - 1];               \
        const PairRec &B_ = (a).pairs[bra_];                                    \
        const PairRec &K_ = (a).pairs[ket_];                                    \
        const double wq_ = pair_weight(bra_, ket_, B_, K_);                     \
        screen_quartet((a), B_, K_, valid_);                                    \
        const int n_ = count_selected(valid_ && sl == 0);                       \
        add_count((a), n_);                                                     \
        if (n_ > 0) k2_body<LI, LJ, LK, LL, R, MODE_JK>((a), tabs, dig, bra_, ket_, valid_, wq_, 0); \
    } while (0)

template <int LI, int LJ, int LK, int LL, typename R, int MODE>
__global__ void __launch_bounds__(64) jk_k2(const JkArgs a) {
    using F = K2Cfg<LI, LJ, LK, LL>;
    constexpr int QW = F::QW, LPQ = F::LPQ;
    __shared__ R tabs[QW * F::TAB];
    __shared__ double dig[F::DIGW];
    const int lane = threadIdx.x;
    const int q = QW > 1 ? lane / LPQ : 0;
    const int sl = QW > 1 ? lane % LPQ : lane;
    const bool lane_used = q < QW;
    const int qq = lane_used ? q : 0;
    if constexpr (MODE == MODE_JK) {
        JK_K2_TILE(a, (int)blockIdx.x);
    } else {
        const int gq = blockIdx.x * QW + qq;
        const bool valid = lane_used && gq < a.nq;
        const int gg = gq < a.nq ? gq : a.nq - 1;
        k2_body<LI, LJ, LK, LL, R, MODE_EXPORT>(a, tabs, dig, a.q_bra[gg], a.q_ket[gg], valid, 1.0, gq);
    }
}

// Row mode for family 2: four independent waves per workgroup walk one bra's
// ket prefix (interleaved by QW quartets), sharing the bra's K rows and J_IJ
// in LDS; one workgroup barrier before the final flush.
// Dynamic LDS: [nset][(NI+NJ) ncols + NI NJ] doubles, then (waves) x
// DIGW doubles, then (waves) x QW x TAB reals.
template <int LI, int LJ, int LK, int LL>
struct K2RowLds {
    using F = K2Cfg<LI, LJ, LK, LL>;
    // per wave of the workgroup
    template <typename R>
    static constexpr size_t fixed() { return (size_t)F::DIGW * sizeof(double) + (size_t)F::QW * F::TAB * sizeof(R); }
    static constexpr size_t per_set(int ncols) {
        return sizeof(double) * ((size_t)(ncart(LI) + ncart(LJ)) * ncols + (size_t)ncart(LI) * ncart(LJ));
    }
};

// (The body stays in the kernel itself: behind one more inlined function
// layer hipcc moved the (ff|ff) FP64 accumulators to scratch and the kernel
// returned wrong values, as with the tile prologue.)
template <int LI, int LJ, int LK, int LL, typename R, int NT, bool BATCH>
__global__ void __launch_bounds__(NT) jk_k2_row(const JkArgs a_in, const BatchDesc *__restrict__ descs, int ndesc) {
    using C = Cls<LI, LJ, LK, LL>;
    using F = K2Cfg<LI, LJ, LK, LL>;
    constexpr int NI = C::NI, NJ = C::NJ, NAB = C::NAB;
    constexpr int QW = F::QW, LPQ = F::LPQ, NW = NT / 64;
    extern __shared__ double smem2[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = lane_index();
    int task = blockIdx.x, m = 0;
    if constexpr (BATCH) {
        m = __builtin_amdgcn_readfirstlane(batch_desc(descs, ndesc, task));
        task -= descs[m].tile_base;
    }
    const JkArgs &a = BATCH ? desc_args(descs, m) : a_in;
    const int ncols = a.ncolK + (a.seg_same ? 0 : a.ncolL);
    const int segL = a.seg_same ? 0 : a.ncolK;
    const int per_set = (NI + NJ) * ncols + NAB;
    double *rows = smem2;
    double *dig = rows + (size_t)per_set * a.nset + (size_t)wave * F::DIGW;
    R *tabs = (R *)(rows + (size_t)per_set * a.nset + NW * F::DIGW) + (size_t)wave * QW * F::TAB;
    const int i = a.row_pos[3 * task];
    const int jbeg = a.row_pos[3 * task + 1], cnt = a.row_pos[3 * task + 2];
    const int bra = a.bra_list[i];
    // a task none of whose quartets can be selected ends here (uniform in the workgroup)
    if (!prefix_selectable(a, a.pairs[bra].q, a.pairs[a.ket_list[jbeg]].q)) return;
    for (int t = tid; t < per_set * a.nset; t += NT) rows[t] = 0.0;
    __syncthreads();
    const int q = QW > 1 ? lane / LPQ : 0;
    const int sl = QW > 1 ? lane % LPQ : lane;
    const bool lane_used = q < QW;
    const int qq = lane_used ? q : 0;
    const PairRec &B = a.pairs[bra];
    int evaluated = 0;  // quartets this wave evaluated (wave-uniform)
    for (int j0 = jbeg + wave * QW; j0 < cnt; j0 += NW * QW) {
        if (!prefix_selectable(a, B.q, a.pairs[a.ket_list[j0]].q)) break;  // uniform in the wave
        const int j = j0 + qq;
        bool valid = lane_used && j < cnt;
        const int ket = a.ket_list[j < cnt ? j : cnt - 1];
        const PairRec &Kt = a.pairs[ket];
        const double wq = pair_weight(bra, ket, B, Kt);
        screen_quartet(a, B, Kt, valid);
        // (no workgroup barrier inside this loop: a wave may skip a step)
        const int nv = count_selected(valid && sl == 0);
        if (nv == 0) continue;
        evaluated += nv;
        k2_body<LI, LJ, LK, LL, R, MODE_JK, true>(a, tabs, dig, bra, ket, valid, wq, 0, rows, ncols, segL);
    }
    add_count(a, evaluated);
    __syncthreads();
    const int n = a.nao;
    for (int s = 0; s < a.nset; ++s) {
        const double *rm = rows + s * per_set;
        double *Jm = a.J + s * a.mstride;
        double *Km = a.K + s * a.mstride;
        for (int t = tid; t < per_set; t += NT) {
            const double v = rm[t];
            if (v == 0.0) continue;
            if (t >= (NI + NJ) * ncols) {
                const int e = t - (NI + NJ) * ncols;
                atomic_add_f64(&Jm[(B.aoi + e / NJ) * n + B.aoj + e % NJ], v);
                continue;
            }
            const int r = t / ncols, c = t % ncols;
            const int row = r < NI ? B.aoi + r : B.aoj + (r - NI);
            int col;
            if (c < a.ncolK) col = a.aoc[a.tshK[c / ncart(LK)]] + c % ncart(LK);
            else col = a.aoc[a.tshL[(c - a.ncolK) / ncart(LL)]] + (c - a.ncolK) % ncart(LL);
            atomic_add_f64(&Km[row * n + col], v);
        }
    }
}


// ===========================================================================
// Family 3: a lane group per quartet, one lane per Cartesian component a of
// the bra's first shell; each lane keeps the block (a b | c d) for all b, c,
// d in registers.  Per primitive quartet the lanes of a group first evaluate
// the roots and weights (one lane per root) and then the vertical
// recurrence tables G(n, m) of every root and direction (one lane per
// table) into LDS; each lane then reads the rows n = a_x .. a_x + l_J of
// its own component, applies the horizontal transfers on the bra and the
// ket in registers and accumulates its elements.  Only the small G tables
// pass through LDS, once per lane and root, instead of three table reads
// per element and root.  Row mode only: the workgroup walks a chunk of one
// bra's kets and keeps the bra's K rows and J_IJ in LDS (flushed once);
// J'_KL of each quartet goes to the pair-ordered buffer.
// ===========================================================================
template <int LI, int LJ, int LK, int LL>
struct K3Cfg {
    using C = Cls<LI, LJ, LK, LL>;
    static constexpr int NA = LI + LJ, NCC = LK + LL;
    static constexpr int GS = (NA + 1) * (NCC + 1);   // G entries per (root, direction)
    static constexpr int ROWS = (LJ + 1) * (NCC + 1); // G entries one lane reads per (root, direction)
    static constexpr int LPQ = C::NI;                 // lanes per quartet
    static constexpr int QW = 64 / LPQ;               // quartets per wave
    static constexpr int NV = C::NJ * C::NK * C::NL;  // accumulators per lane
    static constexpr int TS = (LJ + 1) * (LK + 1) * (LL + 1);  // per-lane table per direction
    // primitive quartets whose tables are built at once: enough that most
    // lanes of a quartet's group have a (primitive, root) task, within
    // 20 KB of tables per wave (in FP64)
    static constexpr int pb_() {
        int pb = LPQ / C::NR;
        const int cap = (20 * 1024) / (QW * C::NR * 3 * GS * 8);
        if (pb > cap) pb = cap;
        return pb < 1 ? 1 : pb;
    }
    static constexpr int PB = pb_();
    // one quartet's tables, [PB][NR][3][GS], padded to an odd number of
    // elements so the quartets of a wave start on different LDS banks
    // (measured on the 32-water TZ set: family-3 rows 120.4 -> 114.4 ms in
    // FP64, 95.2 -> 87.7 ms in FP32)
    static constexpr int GQ = PB * C::NR * 3 * GS + ((PB * C::NR * 3 * GS) % 2 == 0 ? 1 : 0);
    // per wave, in R: G [QW][GQ]
    static constexpr int GW = QW * GQ;
    // per wave, doubles: J'_KL of the wave's quartets [QW][NK NL]
    static constexpr int JW = QW * C::NK * C::NL;
    template <typename R>
    static constexpr size_t wave_bytes() { return (size_t)JW * sizeof(double) + (size_t)GW * sizeof(R); }
    static constexpr size_t per_set(int ncols) {
        return sizeof(double) * ((size_t)(C::NI + C::NJ) * ncols + (size_t)C::NI * C::NJ);
    }
};

// Vertical recurrence of one direction and root: G(n, m), n <= NA, m <= NC,
// scaled by s, stored row-major [n][m] at dst.
template <int NA, int NC, typename R>
__device__ __forceinline__ void vrr2d(R c00, R c00p, R b00, R b10, R b01, R s, R *dst) {
    R G[NA + 1][NC + 1];
    G[0][0] = s;
    if constexpr (NA > 0) G[1][0] = c00 * s;
#pragma unroll
    for (int n = 1; n < NA; ++n) G[n + 1][0] = c00 * G[n][0] + (R)n * b10 * G[n - 1][0];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
#pragma unroll
        for (int n = 0; n <= NA; ++n) {
            R v = c00p * G[n][m];
            if (m > 0) v += (R)m * b01 * G[n][m - 1];
            if (n > 0) v += (R)n * b00 * G[n - 1][m];
            G[n][m + 1] = v;
        }
    }
#pragma unroll
    for (int n = 0; n <= NA; ++n)
#pragma unroll
        for (int m = 0; m <= NC; ++m) dst[n * (NC + 1) + m] = G[n][m];
}

// One lane's table T[b][c][d] (b <= LJ, c <= LK, d <= LL) of one direction
// from the G rows n = a .. a + LJ (src, [LJ + 1][NC + 1]): horizontal
// transfer on the bra with ab, then on the ket with cd.
template <int LJ, int LK, int LL, typename R>
__device__ __forceinline__ void hrr_lane(const R *src, R ab, R cd, R (&T)[(LJ + 1) * (LK + 1) * (LL + 1)]) {
    constexpr int NC = LK + LL;
    R X[LJ + 1][NC + 1];
#pragma unroll
    for (int k = 0; k <= LJ; ++k)
#pragma unroll
        for (int m = 0; m <= NC; ++m) X[k][m] = src[k * (NC + 1) + m];
#pragma unroll
    for (int b = 0; b <= LJ; ++b) {
        if (b > 0) {
#pragma unroll
            for (int k = 0; k <= LJ - b; ++k)
#pragma unroll
                for (int m = 0; m <= NC; ++m) X[k][m] = X[k + 1][m] + ab * X[k][m];
        }
        R Y[NC + 1];
#pragma unroll
        for (int m = 0; m <= NC; ++m) Y[m] = X[0][m];
#pragma unroll
        for (int d = 0; d <= LL; ++d) {
            if (d > 0) {
#pragma unroll
                for (int c = 0; c <= NC - d; ++c) Y[c] = Y[c + 1] + cd * Y[c];
            }
#pragma unroll
            for (int c = 0; c <= LK; ++c) T[(b * (LK + 1) + c) * (LL + 1) + d] = Y[c];
        }
    }
}

template <int LI, int LJ, int LK, int LL, typename R, int NT, bool BATCH>
__global__ void __launch_bounds__(NT) jk_k3_row(const JkArgs a_in, const BatchDesc *__restrict__ descs, int ndesc) {
    using C = Cls<LI, LJ, LK, LL>;
    using F = K3Cfg<LI, LJ, LK, LL>;
    constexpr int NI = C::NI, NJ = C::NJ, NK = C::NK, NL = C::NL, NR = C::NR, NAB = C::NAB;
    constexpr int LPQ = F::LPQ, QW = F::QW, NW = NT / 64, NCC = F::NCC, TS = F::TS, PB = F::PB;
    extern __shared__ double smem3[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = lane_index();
    int task = blockIdx.x, m = 0;
    if constexpr (BATCH) {
        m = __builtin_amdgcn_readfirstlane(batch_desc(descs, ndesc, task));
        task -= descs[m].tile_base;
    }
    const JkArgs &a = BATCH ? desc_args(descs, m) : a_in;
    const int ncols = a.ncolK + (a.seg_same ? 0 : a.ncolL);
    const int segL = a.seg_same ? 0 : a.ncolK;
    const int per_set = (NI + NJ) * ncols + NAB;
    double *rows = smem3;
    double *jkl = rows + (size_t)per_set * a.nset + (size_t)wave * F::JW;
    R *gt = (R *)(rows + (size_t)per_set * a.nset + (size_t)NW * F::JW) + (size_t)wave * F::GW;
    const int i = a.row_pos[3 * task];
    const int jbeg = a.row_pos[3 * task + 1], cnt = a.row_pos[3 * task + 2];
    const int bra = a.bra_list[i];
    // a task none of whose quartets can be selected ends here (uniform in the workgroup)
    if (!prefix_selectable(a, a.pairs[bra].q, a.pairs[a.ket_list[jbeg]].q)) return;
    for (int t = tid; t < per_set * a.nset; t += NT) rows[t] = 0.0;
    for (int t = lane; t < F::JW; t += 64) jkl[t] = 0.0;
    __syncthreads();
    const int q = lane / LPQ, ia = lane % LPQ;
    const bool lane_used = q < QW;
    const int qq = lane_used ? q : 0;
    // Cartesian exponents of this lane's bra component
    int ae[3] = {0, 0, 0};
#pragma unroll
    for (int t = 0; t < NI; ++t)
        if (t == ia) { ae[0] = cart_comp(LI, t, 0); ae[1] = cart_comp(LI, t, 1); ae[2] = cart_comp(LI, t, 2); }
    const PairRec B = a.pairs[bra];
    const R ab[3] = {(R)B.ab[0], (R)B.ab[1], (R)B.ab[2]};
    const int n = a.nao;
    int evaluated = 0;  // quartets this wave evaluated (wave-uniform)
    for (int j0 = jbeg + wave * QW; j0 < cnt; j0 += NW * QW) {
        if (!prefix_selectable(a, B.q, a.pairs[a.ket_list[j0]].q)) break;  // uniform in the wave
        const int j = j0 + qq;
        bool valid = lane_used && j < cnt;
        const int ket = a.ket_list[j < cnt ? j : cnt - 1];
        const PairRec Kt = a.pairs[ket];
        const double wq = pair_weight(bra, ket, B, Kt);
        screen_quartet(a, B, Kt, valid);
        // (no workgroup barrier inside this loop: a wave may skip a step)
        const int nv = count_selected(valid && ia == 0);
        if (nv == 0) continue;
        evaluated += nv;
        const R cd[3] = {(R)Kt.ab[0], (R)Kt.ab[1], (R)Kt.ab[2]};
        R V[F::NV];
#pragma unroll
        for (int e = 0; e < F::NV; ++e) V[e] = (R)0;
        const int vb = variant_begin(a.omega), nvar = variant_end(a.omega) - vb;
        const int nit = a.npb * a.npk * nvar;
        R *gq = gt + qq * F::GQ;
        for (int it0 = 0; it0 < nit; it0 += PB) {
            wave_sync();
            // one lane per (primitive quartet of the batch, root): the root
            // and weight, then the vertical recurrence tables of the three
            // directions
            for (int t = ia; t < PB * NR && lane_used; t += LPQ) {
                const int p = t / NR, r = t - p * NR;
                const int it = it0 + p;
                if (it >= nit) break;
                const int ipq = it / nvar, var = vb + it % nvar;
                const int ib = ipq % a.npb, ik = ipq / a.npb;
                const PQuart<R> g = prim_quartet<R>(a.pp[B.pp_off + ib * B.pp_stride], a.pp[Kt.pp_off + ik * Kt.pp_stride]);
                R u, w;
                rys_root1_op<NR, R>(g.T, g.rho, a.omega, var, r, a.tab, u, w);
                const R b00 = (R)0.5 * u * g.rpq;
                const R b10 = g.hb * ((R)1 - g.fq * u);
                const R b01 = g.hk * ((R)1 - g.fp * u);
                R *dst = gq + (p * NR + r) * 3 * F::GS;
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const R c00 = g.PA[x] - g.fq * u * g.PQ[x];
                    const R c00p = g.QC[x] + g.fp * u * g.PQ[x];
                    vrr2d<F::NA, NCC, R>(c00, c00p, b00, b10, b01, x == 2 ? w * g.pref : (R)1, dst + x * F::GS);
                }
            }
            wave_sync();
            // this lane's rows, transfers and elements, primitive quartet by
            // primitive quartet and root by root
            for (int p = 0; p < PB; ++p) {
                if (it0 + p >= nit) break;  // uniform in the wave
                const R *gp = gq + p * NR * 3 * F::GS;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    R T0[TS], T1[TS], T2[TS];
                    hrr_lane<LJ, LK, LL, R>(gp + (r * 3 + 0) * F::GS + ae[0] * (NCC + 1), ab[0], cd[0], T0);
                    hrr_lane<LJ, LK, LL, R>(gp + (r * 3 + 1) * F::GS + ae[1] * (NCC + 1), ab[1], cd[1], T1);
                    hrr_lane<LJ, LK, LL, R>(gp + (r * 3 + 2) * F::GS + ae[2] * (NCC + 1), ab[2], cd[2], T2);
#pragma unroll
                    for (int b = 0; b < NJ; ++b)
#pragma unroll
                        for (int c = 0; c < NK; ++c)
#pragma unroll
                            for (int d = 0; d < NL; ++d) {
                                const int ix = (cart_comp(LJ, b, 0) * (LK + 1) + cart_comp(LK, c, 0)) * (LL + 1) + cart_comp(LL, d, 0);
                                const int iy = (cart_comp(LJ, b, 1) * (LK + 1) + cart_comp(LK, c, 1)) * (LL + 1) + cart_comp(LL, d, 1);
                                const int iz = (cart_comp(LJ, b, 2) * (LK + 1) + cart_comp(LK, c, 2)) * (LL + 1) + cart_comp(LL, d, 2);
                                V[(b * NK + c) * NL + d] += T0[ix] * T1[iy] * T2[iz];
                            }
                }
            }
        }
        // digestion of this lane's elements (a b | c d), b, c, d all
        const int cK = a.tpos[Kt.ish] * NK, cL = segL + a.tpos[Kt.jsh] * NL;
        const int ga = B.aoi + ia;
        for (int s = 0; s < a.nset; ++s) {
            const double *D = a.D + s * a.mstride;
            double *rm = rows + s * per_set;
            double *rI = rm, *rJ = rm + NI * ncols, *rjij = rm + (NI + NJ) * ncols;
            if (valid) {
                if (a.do_j) {
                    double dab[NJ], jab[NJ];
#pragma unroll
                    for (int b = 0; b < NJ; ++b) {
                        dab[b] = D[ga * n + B.aoj + b];
                        jab[b] = 0.0;
                    }
#pragma unroll
                    for (int c = 0; c < NK; ++c)
#pragma unroll
                        for (int d = 0; d < NL; ++d) {
                            const double dcd = D[(Kt.aoi + c) * n + Kt.aoj + d];
                            double p = 0.0;
#pragma unroll
                            for (int b = 0; b < NJ; ++b) {
                                const double v = (double)V[(b * NK + c) * NL + d];
                                jab[b] += v * dcd;
                                p += v * dab[b];
                            }
                            atomicAdd(&jkl[qq * (NK * NL) + c * NL + d], 2.0 * wq * p);
                        }
#pragma unroll
                    for (int b = 0; b < NJ; ++b) atomicAdd(&rjij[ia * NJ + b], 2.0 * wq * jab[b]);
                }
                if (a.do_k) {
                    double dac[NK], dad[NL];
#pragma unroll
                    for (int c = 0; c < NK; ++c) dac[c] = D[ga * n + Kt.aoi + c];
#pragma unroll
                    for (int d = 0; d < NL; ++d) dad[d] = D[ga * n + Kt.aoj + d];
                    double kac[NK], kad[NL];
#pragma unroll
                    for (int c = 0; c < NK; ++c) kac[c] = 0.0;
#pragma unroll
                    for (int d = 0; d < NL; ++d) kad[d] = 0.0;
#pragma unroll
                    for (int b = 0; b < NJ; ++b) {
                        const int gb = B.aoj + b;
                        double kbc[NK], kbd[NL];
#pragma unroll
                        for (int c = 0; c < NK; ++c) kbc[c] = 0.0;
#pragma unroll
                        for (int d = 0; d < NL; ++d) kbd[d] = 0.0;
#pragma unroll
                        for (int c = 0; c < NK; ++c) {
                            const double dbc = D[gb * n + Kt.aoi + c];
#pragma unroll
                            for (int d = 0; d < NL; ++d) {
                                const double v = (double)V[(b * NK + c) * NL + d];
                                const double dbd = D[gb * n + Kt.aoj + d];
                                kac[c] += v * dbd;
                                kad[d] += v * dbc;
                                kbc[c] += v * dad[d];
                                kbd[d] += v * dac[c];
                            }
                        }
#pragma unroll
                        for (int c = 0; c < NK; ++c) atomicAdd(&rJ[b * ncols + cK + c], wq * kbc[c]);
#pragma unroll
                        for (int d = 0; d < NL; ++d) atomicAdd(&rJ[b * ncols + cL + d], wq * kbd[d]);
                    }
#pragma unroll
                    for (int c = 0; c < NK; ++c) atomicAdd(&rI[ia * ncols + cK + c], wq * kac[c]);
#pragma unroll
                    for (int d = 0; d < NL; ++d) atomicAdd(&rI[ia * ncols + cL + d], wq * kad[d]);
                }
            }
            if (a.do_j) {
                // J'_KL of the wave's quartets into the pair-ordered buffer
                wave_sync();
                for (int t = lane; t < QW * NK * NL; t += 64) {
                    const int q2 = t / (NK * NL), e = t % (NK * NL);
                    const double v = jkl[t];
                    jkl[t] = 0.0;
                    const int j2 = j0 + q2;
                    if (j2 < cnt && v != 0.0) {
                        const PairRec &K2 = a.pairs[a.ket_list[j2]];
                        atomic_add_f64(&a.jp[s * a.jpstride + K2.jp_off + (int64_t)e * K2.pp_stride], v);
                    }
                }
                wave_sync();
            }
        }
    }
    add_count(a, evaluated);
    __syncthreads();
    // flush nonzero entries to the global J', K'
    for (int s = 0; s < a.nset; ++s) {
        const double *rm = rows + s * per_set;
        double *Jm = a.J + s * a.mstride;
        double *Km = a.K + s * a.mstride;
        for (int t = tid; t < per_set; t += NT) {
            const double v = rm[t];
            if (v == 0.0) continue;
            if (t >= (NI + NJ) * ncols) {
                const int e = t - (NI + NJ) * ncols;
                atomic_add_f64(&Jm[(B.aoi + e / NJ) * n + B.aoj + e % NJ], v);
                continue;
            }
            const int r = t / ncols, c = t % ncols;
            const int row = r < NI ? B.aoi + r : B.aoj + (r - NI);
            int col;
            if (c < a.ncolK) col = a.aoc[a.tshK[c / NK]] + c % NK;
            else col = a.aoc[a.tshL[(c - a.ncolK) / NL]] + (c - a.ncolK) % NL;
            atomic_add_f64(&Km[row * n + col], v);
        }
    }
}

// ===========================================================================
// Batched builds: one launch per (class, family) covers the tiles of every
// molecule of the batch.  Global tile g belongs to the descriptor m with
// tile_base[m] <= g < tile_base[m + 1]; each descriptor holds the JkArgs of
// one (molecule, class task), heaviest first, so the dispatcher hands out
// the long tiles early.
// ===========================================================================
template <int LI, int LJ, int LK, int LL, typename R>
__global__ void __launch_bounds__(256) jk_k1_batch(const BatchDesc *__restrict__ descs, int ndesc, int total) {
    const int g = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (g >= total) return;
    const int m = __builtin_amdgcn_readfirstlane(batch_desc(descs, ndesc, g));
    k1_tile<LI, LJ, LK, LL, R>(desc_args(descs, m), g - descs[m].tile_base);
}

template <int LI, int LJ, int LK, int LL, typename R>
__global__ void __launch_bounds__(64) jk_k2_batch(const BatchDesc *__restrict__ descs, int ndesc, int total) {
    using F = K2Cfg<LI, LJ, LK, LL>;
    constexpr int QW = F::QW, LPQ = F::LPQ;
    __shared__ R tabs[QW * F::TAB];
    __shared__ double dig[F::DIGW];
    const int lane = threadIdx.x;
    const int q = QW > 1 ? lane / LPQ : 0;
    const int sl = QW > 1 ? lane % LPQ : lane;
    const bool lane_used = q < QW;
    const int qq = lane_used ? q : 0;
    const int g = blockIdx.x;
    const int m = __builtin_amdgcn_readfirstlane(batch_desc(descs, ndesc, g));
    const JkArgs &a = desc_args(descs, m);
    JK_K2_TILE(a, g - descs[m].tile_base);
}

}  // namespace jk
