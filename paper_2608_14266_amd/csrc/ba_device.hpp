// Device-side helpers shared by the gfx950 kernels of libba.
// Wave64 reductions, double-double error-free transforms, small 3x3 algebra.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BA_WAVE 64

namespace ba {

// ---------------------------------------------------------------- wave reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, BA_WAVE);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, BA_WAVE));
    return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, BA_WAVE));
    return v;
}

// Block-wide reductions for blocks of 64 * NW threads: wave reductions, then
// the wave results combined in wave order by every thread (fixed order, so
// deterministic).  `lds` holds NW entries; the block synchronises twice.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; i++) s += lds[i];
    __syncthreads();
    return s;
}

template <int NW>
__device__ __forceinline__ double block_max(double v, double *lds) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = lds[0];
#pragma unroll
    for (int i = 1; i < NW; i++) s = fmax(s, lds[i]);
    __syncthreads();
    return s;
}

// Several block reductions behind one barrier: each value is reduced exactly
// as block_sum / block_max / block_min_i reduce it (same wave order, so the
// results are bitwise those of the separate calls).  The block synchronises
// once; the caller synchronises again before it writes these LDS arrays anew.
template <int NW>
__device__ __forceinline__ void block_sum_max(double &s, double &m, double *lds_s, double *lds_m) {
    s = wave_sum(s);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) {
        lds_s[threadIdx.x >> 6] = s;
        lds_m[threadIdx.x >> 6] = m;
    }
    __syncthreads();
    double a = 0.0, b = lds_m[0];
#pragma unroll
    for (int i = 0; i < NW; i++) a += lds_s[i];
#pragma unroll
    for (int i = 1; i < NW; i++) b = fmax(b, lds_m[i]);
    s = a;
    m = b;
}

template <int NW>
__device__ __forceinline__ void block_sum2_min(double &s0, double &s1, int &k, double *lds_s0, double *lds_s1,
                                               int *lds_k) {
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    k = wave_min_i(k);
    if ((threadIdx.x & 63) == 0) {
        lds_s0[threadIdx.x >> 6] = s0;
        lds_s1[threadIdx.x >> 6] = s1;
        lds_k[threadIdx.x >> 6] = k;
    }
    __syncthreads();
    double a = 0.0, b = 0.0;
    int c = lds_k[0];
#pragma unroll
    for (int i = 0; i < NW; i++) a += lds_s0[i];
#pragma unroll
    for (int i = 0; i < NW; i++) b += lds_s1[i];
#pragma unroll
    for (int i = 1; i < NW; i++) c = min(c, lds_k[i]);
    s0 = a;
    s1 = b;
    k = c;
}

template <int NW>
__device__ __forceinline__ int block_min_i(int v, int *lds) {
    v = wave_min_i(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    int s = lds[0];
#pragma unroll
    for (int i = 1; i < NW; i++) s = min(s, lds[i]);
    __syncthreads();
    return s;
}

// Reduce-scatter of 32 per-lane values over a wave64: after five halving
// exchanges and one final one, lane l holds the sum over all 64 lanes of
// value l / 2 (fixed exchange order, so the result is deterministic).
__device__ __forceinline__ double wave_reduce_scatter32(double (&a)[32], int lane) {
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const bool hi = lane & 32;
        const double mine = hi ? a[16 + i] : a[i], other = hi ? a[i] : a[16 + i];
        a[i] = mine + __shfl_xor(other, 32, BA_WAVE);
    }
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const bool hi = lane & 16;
        const double mine = hi ? a[8 + i] : a[i], other = hi ? a[i] : a[8 + i];
        a[i] = mine + __shfl_xor(other, 16, BA_WAVE);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const bool hi = lane & 8;
        const double mine = hi ? a[4 + i] : a[i], other = hi ? a[i] : a[4 + i];
        a[i] = mine + __shfl_xor(other, 8, BA_WAVE);
    }
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const bool hi = lane & 4;
        const double mine = hi ? a[2 + i] : a[i], other = hi ? a[i] : a[2 + i];
        a[i] = mine + __shfl_xor(other, 4, BA_WAVE);
    }
    {
        const bool hi = lane & 2;
        const double mine = hi ? a[1] : a[0], other = hi ? a[0] : a[1];
        a[0] = mine + __shfl_xor(other, 2, BA_WAVE);
    }
    return a[0] + __shfl_xor(a[0], 1, BA_WAVE);
}

// One halving exchange of a reduce-scatter: lanes with bit W set keep the
// upper W of the live values, the others the lower W, each adding its
// partner's copy (constant trip count, so the array stays in registers).
template <int W>
__device__ __forceinline__ void reduce_scatter_stage(double (&a)[64], int lane) {
    const bool hi = lane & W;
#pragma unroll
    for (int i = 0; i < W; i++) {
        const double mine = hi ? a[W + i] : a[i], other = hi ? a[i] : a[W + i];
        a[i] = mine + __shfl_xor(other, W, BA_WAVE);
    }
}

// Reduce-scatter of 64 per-lane values: after six halving exchanges lane l
// holds the sum over all 64 lanes of value l (fixed order, deterministic).
__device__ __forceinline__ double wave_reduce_scatter64(double (&a)[64], int lane) {
    reduce_scatter_stage<32>(a, lane);
    reduce_scatter_stage<16>(a, lane);
    reduce_scatter_stage<8>(a, lane);
    reduce_scatter_stage<4>(a, lane);
    reduce_scatter_stage<2>(a, lane);
    reduce_scatter_stage<1>(a, lane);
    return a[0];
}

// ---------------------------------------------------------------- error-free transforms
// Knuth TwoSum: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Double-double accumulator (hi, lo) += x.
__device__ __forceinline__ void dd_add(double &hi, double &lo, double x) {
    double s, e;
    two_sum(hi, x, s, e);
    e += lo;
    two_sum(s, e, hi, lo);
}

// (hi, lo) += (bhi, blo)
__device__ __forceinline__ void dd_add_dd(double &hi, double &lo, double bhi, double blo) {
    double s, e;
    two_sum(hi, bhi, s, e);
    e += lo + blo;
    two_sum(s, e, hi, lo);
}

__device__ __forceinline__ void wave_dd_sum(double &hi, double &lo) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double h2 = __shfl_xor(hi, o, BA_WAVE), l2 = __shfl_xor(lo, o, BA_WAVE);
        dd_add_dd(hi, lo, h2, l2);
    }
}

// ---------------------------------------------------------------- 3x3 helpers
__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }

struct Pose {
    double r[9];
    double t[3];
};

__device__ __forceinline__ void load_pose(const double *__restrict__ poses, int j, Pose &p) {
    const double *q = poses + 12 * (int64_t)j;
#pragma unroll
    for (int k = 0; k < 9; k++) p.r[k] = q[k];
#pragma unroll
    for (int k = 0; k < 3; k++) p.t[k] = q[9 + k];
}

// Pose change from a reference pose: E = R R0^T - I and dt = t - t0, so a
// world point x placed by T0 moves to x + E (x - t0) + dt under T.
struct PoseDelta {
    double E[9];
    double dt[3];
};

__device__ __forceinline__ void pose_delta(const Pose &P, const Pose &P0, PoseDelta &D) {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++)
            D.E[3 * i + k] = fma(P.r[3 * i], P0.r[3 * k], fma(P.r[3 * i + 1], P0.r[3 * k + 1],
                                 P.r[3 * i + 2] * P0.r[3 * k + 2])) - (i == k ? 1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < 3; k++) D.dt[k] = P.t[k] - P0.t[k];
}

// D = E S + S E^T + E S E^T for symmetric S (6 unique), so that
// (I + E) S (I + E)^T = S + D with D of the size of E.
template <typename T>
__device__ __forceinline__ void delta_sym(const T *E, const T *S, T *D) {
    const T Sf[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
    T A[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            A[i][j] = fmaT(E[3 * i], Sf[0][j], fmaT(E[3 * i + 1], Sf[1][j], E[3 * i + 2] * Sf[2][j]));
    const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const int i = ii[q], j = jj[q];
        D[q] = A[i][j] + A[j][i] + fmaT(A[i][0], E[3 * j], fmaT(A[i][1], E[3 * j + 1], A[i][2] * E[3 * j + 2]));
    }
}

// y = R x
template <typename T>
__device__ __forceinline__ void rot(const T *r, const T *x, T *y) {
    y[0] = fmaT(r[0], x[0], fmaT(r[1], x[1], r[2] * x[2]));
    y[1] = fmaT(r[3], x[0], fmaT(r[4], x[1], r[5] * x[2]));
    y[2] = fmaT(r[6], x[0], fmaT(r[7], x[1], r[8] * x[2]));
}

// St = R S R^T for symmetric S (6: xx xy xz yy yz zz); output 6 unique.
template <typename T>
__device__ __forceinline__ void rot_sym(const T *r, const T *s, T *o) {
    // M = R S (3x3)
    T m[9];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        m[3 * i + 0] = fmaT(r[3 * i], s[0], fmaT(r[3 * i + 1], s[1], r[3 * i + 2] * s[2]));
        m[3 * i + 1] = fmaT(r[3 * i], s[1], fmaT(r[3 * i + 1], s[3], r[3 * i + 2] * s[4]));
        m[3 * i + 2] = fmaT(r[3 * i], s[2], fmaT(r[3 * i + 1], s[4], r[3 * i + 2] * s[5]));
    }
    // O = M R^T : O_ij = sum_k M_ik R_jk
    o[0] = fmaT(m[0], r[0], fmaT(m[1], r[1], m[2] * r[2]));
    o[1] = fmaT(m[0], r[3], fmaT(m[1], r[4], m[2] * r[5]));
    o[2] = fmaT(m[0], r[6], fmaT(m[1], r[7], m[2] * r[8]));
    o[3] = fmaT(m[3], r[3], fmaT(m[4], r[4], m[5] * r[5]));
    o[4] = fmaT(m[3], r[6], fmaT(m[4], r[7], m[5] * r[8]));
    o[5] = fmaT(m[6], r[6], fmaT(m[7], r[7], m[8] * r[8]));
}

template <typename T>
__device__ __forceinline__ void cross(const T *a, const T *b, T *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T>
__device__ __forceinline__ T dot(const T *a, const T *b) {
    return fmaT(a[0], b[0], fmaT(a[1], b[1], a[2] * b[2]));
}

// symmetric (6) times vector
template <typename T>
__device__ __forceinline__ void sym_mv(const T *s, const T *x, T *y) {
    y[0] = fmaT(s[0], x[0], fmaT(s[1], x[1], s[2] * x[2]));
    y[1] = fmaT(s[1], x[0], fmaT(s[3], x[1], s[4] * x[2]));
    y[2] = fmaT(s[2], x[0], fmaT(s[4], x[1], s[5] * x[2]));
}

// ---------------------------------------------------------------- 3x3 symmetric eigen
// Smallest eigenpair of a symmetric positive semi-definite 3x3 (6 unique).
// Cyclic Jacobi rotations (Golub & Van Loan, Sec. 8.5) with a fixed sweep
// budget and an early exit once every off-diagonal entry is negligible;
// returns all three eigenvalues ascending in lam and the eigenvector of
// lam[0] in u.
__device__ __forceinline__ void jacobi_rot(double &app, double &aqq, double &apq, double &apr, double &aqr,
                                           double *vp, double *vq) {
    // annihilate apq; r is the remaining index.
    if (apq == 0.0) return;
    double theta = (aqq - app) / (2.0 * apq);
    double t = (fabs(theta) > 1e150) ? 0.5 / theta
                                     : copysign(1.0, theta) / (fabs(theta) + sqrt(fma(theta, theta, 1.0)));
    double c = 1.0 / sqrt(fma(t, t, 1.0));
    double s = t * c;
    double tau = s / (1.0 + c);
    double napp = app - t * apq;
    double naqq = aqq + t * apq;
    double r1 = apr - s * (aqr + tau * apr);
    double r2 = aqr + s * (apr - tau * aqr);
    app = napp; aqq = naqq; apq = 0.0; apr = r1; aqr = r2;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        double a = vp[k], b = vq[k];
        vp[k] = a - s * (b + tau * a);
        vq[k] = b + s * (a - tau * b);
    }
}

__device__ __forceinline__ void eig_sym3(const double *A, double *lam, double *u) {
    double a00 = A[0], a01 = A[1], a02 = A[2], a11 = A[3], a12 = A[4], a22 = A[5];
    double v0[3] = {1, 0, 0}, v1[3] = {0, 1, 0}, v2[3] = {0, 0, 1};
    for (int sweep = 0; sweep < 12; sweep++) {
        double scale = fabs(a00) + fabs(a11) + fabs(a22);
        double off = fabs(a01) + fabs(a02) + fabs(a12);
        if (off <= 1e-22 * scale || off == 0.0) break;
        // (0,1), remaining 2
        jacobi_rot(a00, a11, a01, a02, a12, v0, v1);
        // (0,2), remaining 1
        jacobi_rot(a00, a22, a02, a01, a12, v0, v2);
        // (1,2), remaining 0
        jacobi_rot(a11, a22, a12, a01, a02, v1, v2);
    }
    // ascending order
    double d[3] = {a00, a11, a22};
    int i0 = 0, i1 = 1, i2 = 2;
    if (d[i1] < d[i0]) { int t = i0; i0 = i1; i1 = t; }
    if (d[i2] < d[i1]) { int t = i1; i1 = i2; i2 = t; }
    if (d[i1] < d[i0]) { int t = i0; i0 = i1; i1 = t; }
    lam[0] = d[i0]; lam[1] = d[i1]; lam[2] = d[i2];
    const double *vs = (i0 == 0) ? v0 : (i0 == 1 ? v1 : v2);
    u[0] = vs[0]; u[1] = vs[1]; u[2] = vs[2];
}

// Adjugate (cofactor matrix) of a symmetric 3x3 (6 unique), same layout.  For
// B = A - x I with eigenpairs (l_k - x, u_k), adj(B) = sum_k prod_{l != k}
// (l_l - x) u_k u_k^T: as x approaches the smallest eigenvalue its columns all
// turn towards u_0.
__device__ __forceinline__ void adj_sym3(double a00, double a01, double a02, double a11, double a12, double a22,
                                         double *c) {
    c[0] = fma(a11, a22, -a12 * a12);
    c[1] = fma(a02, a12, -a01 * a22);
    c[2] = fma(a01, a12, -a02 * a11);
    c[3] = fma(a00, a22, -a02 * a02);
    c[4] = fma(a01, a02, -a00 * a12);
    c[5] = fma(a00, a11, -a01 * a01);
}

// 1/sqrt(x) for x > 0: the hardware estimate (about half the FP64 mantissa)
// and two Newton steps, which bring it to a few ulp (used to normalise
// vectors, whose unit length the convergence test below relies on).
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y * fma(-0.5 * x * y, y, 1.5);
}

// Smallest eigenpair of a symmetric positive semi-definite 3x3 (6 unique).
//  1. Newton's method on the characteristic polynomial p(x) = det(A - x I),
//     started at x = 0: for a cubic with real roots that starts below the
//     smallest root, the iterates rise monotonically towards it (p is convex
//     there), so the shift approaches lambda_0 from below whatever the
//     spacing of the other two.
//  2. u = the largest column of adj(A - x I), normalised.
//  3. Rayleigh quotient iteration (Parlett, The Symmetric Eigenvalue
//     Problem, Ch. 4) with the inverse step taken as adj(A - s I) u,
//     s = u^T A u, until two iterates agree to rounding.
//  4. lambda_0 = u^T A u; its absolute error is of order eps ||A||, as for
//     any backward-stable method.
// Returns false (and leaves lam0/u unspecified) when the matrix has rank
// below two (lambda_0 = lambda_1 = 0) or the iteration did not end at the
// smallest eigenvalue; the caller then takes the Jacobi path.
__device__ __forceinline__ bool eig_min_sym3(const double *A, double &lam0, double *u) {
    const double a00 = A[0], a01 = A[1], a02 = A[2], a11 = A[3], a12 = A[4], a22 = A[5];
    double c[6];
    adj_sym3(a00, a01, a02, a11, a12, a22, c);
    const double c2 = a00 + a11 + a22;        // trace
    const double c1 = c[0] + c[3] + c[5];     // sum of the principal 2x2 minors
    const double c0 = fma(a00, c[0], fma(a01, c[1], a02 * c[2]));   // determinant
    if (!(c1 > 1e-28 * c2 * c2)) return false;
    double x = 0.0;
    for (int it = 0; it < 40; it++) {
        const double p = fma(-x, fma(-x, c2 - x, c1), c0);    // c0 - x (c1 - x (c2 - x))
        const double dp = fma(x, fma(-3.0, x, 2.0 * c2), -c1);
        const double dx = -p / dp;
        x += dx;
        if (!(fabs(dx) > 1e-4 * x)) break;
    }
    double b[6];
    adj_sym3(a00 - x, a01, a02, a11 - x, a12, a22 - x, b);
    {
        const double n0 = fma(b[0], b[0], fma(b[1], b[1], b[2] * b[2]));
        const double n1 = fma(b[1], b[1], fma(b[3], b[3], b[4] * b[4]));
        const double n2 = fma(b[2], b[2], fma(b[4], b[4], b[5] * b[5]));
        double v0 = b[0], v1 = b[1], v2 = b[2], nn = n0;
        if (n1 > nn) { v0 = b[1]; v1 = b[3]; v2 = b[4]; nn = n1; }
        if (n2 > nn) { v0 = b[2]; v1 = b[4]; v2 = b[5]; nn = n2; }
        if (!(nn > 0.0)) return false;
        const double r = rsqrt_nr(nn);
        u[0] = v0 * r; u[1] = v1 * r; u[2] = v2 * r;
    }
    bool conv = false;
    for (int it = 0; it < 6; it++) {
        const double au0 = fma(a00, u[0], fma(a01, u[1], a02 * u[2]));
        const double au1 = fma(a01, u[0], fma(a11, u[1], a12 * u[2]));
        const double au2 = fma(a02, u[0], fma(a12, u[1], a22 * u[2]));
        const double s = fma(u[0], au0, fma(u[1], au1, u[2] * au2));
        adj_sym3(a00 - s, a01, a02, a11 - s, a12, a22 - s, b);
        const double x0 = fma(b[0], u[0], fma(b[1], u[1], b[2] * u[2]));
        const double x1 = fma(b[1], u[0], fma(b[3], u[1], b[4] * u[2]));
        const double x2 = fma(b[2], u[0], fma(b[4], u[1], b[5] * u[2]));
        const double nn = fma(x0, x0, fma(x1, x1, x2 * x2));
        if (!(nn > 0.0)) {   // u is an exact eigenvector of the rounded matrix
            conv = true;
            break;
        }
        const double r = rsqrt_nr(nn);
        const double y0 = x0 * r, y1 = x1 * r, y2 = x2 * r;
        const double cs = fabs(fma(y0, u[0], fma(y1, u[1], y2 * u[2])));
        u[0] = y0; u[1] = y1; u[2] = y2;
        if (cs >= 1.0 - 4.0 * 2.220446049250313e-16) {
            conv = true;
            break;
        }
    }
    const double au0 = fma(a00, u[0], fma(a01, u[1], a02 * u[2]));
    const double au1 = fma(a01, u[0], fma(a11, u[1], a12 * u[2]));
    const double au2 = fma(a02, u[0], fma(a12, u[1], a22 * u[2]));
    const double l = fma(u[0], au0, fma(u[1], au1, u[2] * au2));
    // the other two eigenvalues are the roots of y^2 - s2 y + pr with
    // s2 = trace - l and pr = c1 - l s2; l is the smallest iff it lies at or
    // below both (up to rounding of the coefficients)
    const double s2 = c2 - l;
    const double pr = fma(-l, s2, c1);
    const double f = fma(l, l - s2, pr);
    const double tol = 1e-12 * c2;
    if (!conv || f < -tol * c2 || 2.0 * l > s2 + tol) return false;
    lam0 = l;
    return true;
}

// Smallest eigenpair by eig_min_sym3, with the Jacobi iteration for the
// matrices it declines (rank below two, or a pair it cannot separate).
__device__ __forceinline__ void eig_min_sym3_safe(const double *A, double &lam0, double *u) {
    if (!eig_min_sym3(A, lam0, u)) {
        double lam[3];
        eig_sym3(A, lam, u);
        lam0 = lam[0];
    }
}

// All three eigenpairs of the same Jacobi iteration: lam ascending and the
// matching unit eigenvectors U[3 * k .. 3 * k + 2] (k = 0, 1, 2); lam and
// U[0..2] equal eig_sym3's outputs.
__device__ __forceinline__ void eig_sym3_full(const double *A, double *lam, double *U) {
    double a00 = A[0], a01 = A[1], a02 = A[2], a11 = A[3], a12 = A[4], a22 = A[5];
    double v0[3] = {1, 0, 0}, v1[3] = {0, 1, 0}, v2[3] = {0, 0, 1};
    for (int sweep = 0; sweep < 12; sweep++) {
        double scale = fabs(a00) + fabs(a11) + fabs(a22);
        double off = fabs(a01) + fabs(a02) + fabs(a12);
        if (off <= 1e-22 * scale || off == 0.0) break;
        jacobi_rot(a00, a11, a01, a02, a12, v0, v1);
        jacobi_rot(a00, a22, a02, a01, a12, v0, v2);
        jacobi_rot(a11, a22, a12, a01, a02, v1, v2);
    }
    double d[3] = {a00, a11, a22};
    int i0 = 0, i1 = 1, i2 = 2;
    if (d[i1] < d[i0]) { int t = i0; i0 = i1; i1 = t; }
    if (d[i2] < d[i1]) { int t = i1; i1 = i2; i2 = t; }
    if (d[i1] < d[i0]) { int t = i0; i0 = i1; i1 = t; }
    const int ord[3] = {i0, i1, i2};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        lam[k] = d[ord[k]];
        const double *vs = (ord[k] == 0) ? v0 : (ord[k] == 1 ? v1 : v2);
        U[3 * k] = vs[0]; U[3 * k + 1] = vs[1]; U[3 * k + 2] = vs[2];
    }
}

// Exp(phi) as the rotation of the unit quaternion (cos(th/2), sin(th/2) phi/th);
// the ratio sin(th/2)/th uses its Taylor series below 1e-4 rad.
__device__ __forceinline__ void so3_exp(const double *phi, double *E) {
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double w, k;
    if (th2 < 1e-8) {
        w = 1.0 - th2 * (1.0 / 8.0) + th2 * th2 * (1.0 / 384.0);
        k = 0.5 - th2 * (1.0 / 48.0) + th2 * th2 * (1.0 / 3840.0);
    } else {
        const double th = sqrt(th2);
        double sh, chh;
        sincos(0.5 * th, &sh, &chh);
        w = chh;
        k = sh / th;
    }
    const double x = k * phi[0], y = k * phi[1], z = k * phi[2];
    E[0] = 1.0 - 2.0 * (y * y + z * z);
    E[1] = 2.0 * (x * y - z * w);
    E[2] = 2.0 * (x * z + y * w);
    E[3] = 2.0 * (x * y + z * w);
    E[4] = 1.0 - 2.0 * (x * x + z * z);
    E[5] = 2.0 * (y * z - x * w);
    E[6] = 2.0 * (x * z - y * w);
    E[7] = 2.0 * (y * z + x * w);
    E[8] = 1.0 - 2.0 * (x * x + y * y);
}

// T (+) x = (Exp(phi) R, t + dt)
__device__ __forceinline__ void pose_plus(const double *T, const double *x, double *out) {
    double E[9];
    so3_exp(x, E);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            out[3 * i + j] = E[3 * i] * T[j] + E[3 * i + 1] * T[3 + j] + E[3 * i + 2] * T[6 + j];
    out[9] = T[9] + x[3];
    out[10] = T[10] + x[4];
    out[11] = T[11] + x[5];
}

}  // namespace ba
