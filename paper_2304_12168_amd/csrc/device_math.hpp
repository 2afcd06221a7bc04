// Device helpers shared by the kernels of libta: compensated (double-double)
// accumulation, wave-level reductions, XCD-aware block mapping and the
// solution of CTA's auxiliary equation.
#pragma once

#include <math.h>

#include "common.hpp"

namespace ta {

// ---------------------------------------------------------------------------
// compensated accumulation
// ---------------------------------------------------------------------------
struct Acc {
    double p, s;  // value p + s
};

__device__ __forceinline__ void two_sum(double a, double b, double &x, double &y) {
    x = a + b;
    const double z = x - a;
    y = (a - (x - z)) + (b - z);
}

// acc += h + r where h + r is an exact product split (h = fl(a b), r = error)
__device__ __forceinline__ void acc_add_split(Acc &c, double h, double r) {
    double q;
    two_sum(c.p, h, c.p, q);
    c.s = c.s + (q + r);
}

__device__ __forceinline__ void acc_fma(Acc &c, double a, double b) {
    const double h = a * b;
    const double r = __fma_rn(a, b, -h);
    acc_add_split(c, h, r);
}

__device__ __forceinline__ Acc acc_merge(Acc a, Acc b) {
    Acc o;
    double q;
    two_sum(a.p, b.p, o.p, q);
    o.s = (a.s + b.s) + q;
    return o;
}

__device__ __forceinline__ double acc_val(Acc a) { return a.p + a.s; }

template <int W>
__device__ __forceinline__ Acc group_reduce(Acc v) {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) {
        Acc o;
        o.p = __shfl_xor(v.p, off);
        o.s = __shfl_xor(v.s, off);
        v = acc_merge(v, o);
    }
    return v;
}

// Enhanced stop (section 3.2, t >= 2): the first-order iterates
// f_j = F_1(f_{j-1}), f_0 = r, lie in r + span{H r, ..., H^j r}:
// f_j = sum_k c_k H^k r, so f^T H^p f = sum_{k,l} c_k c_l phi_{k+l+p} needs
// phi up to 2j + 2 <= 2t.  a_j = (f^T H f) / (f^T H^2 f); the test is on
// ||A^T f_j||^2 = f^T H f (H = A A^T) or ||A f_j||^2 = f^T H^2 f (H = A);
// x^ = x + sum_i a_{i+1} (A^T) f_i has the coefficients beta_k on the vectors
// the update already uses (A^T H^k r, or H^k r), so the update kernels apply
// x^ as they apply alpha, and r - sum beta_k H^{k+1} r is x^'s residual.
// Returns true at the first j that passes, with beta_0 .. beta_{t-1} set.
__device__ inline bool enhanced_hit(const double *phi, int t, int hmode, double tol_ne_nab,
                                    double *beta) {
    double c[kTMax + 1] = {1.0};
    for (int i = 0; i < t; ++i) beta[i] = 0.0;
    const int ptest = hmode ? 2 : 1;
    for (int j = 1; j < t; ++j) {
        double e1 = 0.0, e2 = 0.0;
        for (int k = 0; k < j; ++k)
            for (int l = 0; l < j; ++l) {
                e1 += c[k] * c[l] * phi[k + l + 1];
                e2 += c[k] * c[l] * phi[k + l + 2];
            }
        if (!(e2 > 0.0) || !isfinite(e1) || !isfinite(e2)) return false;
        const double aj = e1 / e2;
        for (int k = 0; k < j; ++k) beta[k] = fma(aj, c[k], beta[k]);
        for (int k = j; k >= 1; --k) c[k] = fma(-aj, c[k - 1], c[k]);
        double q = 0.0;
        for (int k = 0; k <= j; ++k)
            for (int l = 0; l <= j; ++l) q += c[k] * c[l] * phi[k + l + ptest];
        if (sqrt(fmax(q, 0.0)) <= tol_ne_nab) return true;
    }
    return false;
}

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous
// range of logical blocks so neighbouring rows share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t q = G / 8, rem = G % 8;
    const int64_t x = b % 8, i = b / 8;
    return x * q + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------------------
// The auxiliary equation of CTA (section 3.1, eq. "eqcoeff"), one thread.
// M_ij = phi_{i+j}, g_i = phi_i (i, j = 1..t).  Reading of "minimum-norm
// solution when not unique": ridge solution of an exactly (power-of-two)
// scaled system, continuous in phi.  Steps:
//   order te: t, lowered to i-1 at the first phi_{2i} <= 0;
//   te = 1: alpha_1 = phi_1 / phi_2 (Example 1);
//   else s_i = 2^-floor((e_i - 1)/2) with phi_{2i} = f 2^e_i, f in [0.5, 1);
//        Ms_ij = (phi_{i+j} s_i) s_j, gs_i = phi_i s_i,
//        Ms_ii = fma(Ms_ii, 16 te^2 2^-53, Ms_ii);
//        Cholesky column by column, te lowered to j at a pivot <= 0
//        (te = 1 then uses the closed form);
//        forward / back substitution; alpha_i = s_i alpha~_i.
// ---------------------------------------------------------------------------
// Instantiated per order T with every loop unrolled, so the matrices live in
// registers of the one thread that runs it (te only shrinks, guarded).
template <int T>
__device__ int gram_alpha_t(const double *phi, double *alpha) {
    double s[T], g[T], z[T], at[T];
    double L[T][T];  // scaled matrix, overwritten by its Cholesky factor (lower part)
    int te = T;
#pragma unroll
    for (int i = 0; i < T; ++i) alpha[i] = 0.0;
#pragma unroll
    for (int i = 1; i <= T; ++i) {
        if (te == T && !(phi[2 * i] > 0.0)) te = i - 1;
    }
    if (te <= 0) return 0;
    if (te >= 2) {
#pragma unroll
        for (int i = 0; i < T; ++i) {
            int e = 0;
            (void)frexp(phi[2 * (i + 1)], &e);
            const int kk = (int)floor((e - 1) / 2.0);
            s[i] = ldexp(1.0, -kk);
        }
#pragma unroll
        for (int i = 0; i < T; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j) L[i][j] = (phi[i + j + 2] * s[i]) * s[j];
            g[i] = phi[i + 1] * s[i];
        }
        const double ridge = 16.0 * (double)te * (double)te * ldexp(1.0, -53);
#pragma unroll
        for (int i = 0; i < T; ++i) L[i][i] = __fma_rn(L[i][i], ridge, L[i][i]);
        // Cholesky, column by column; unused columns (j >= te) are skipped
#pragma unroll
        for (int j = 0; j < T; ++j) {
            if (j < te) {
                double d = L[j][j];
#pragma unroll
                for (int k = 0; k < j; ++k) d = __fma_rn(-L[j][k], L[j][k], d);
                if (!(d > 0.0)) {
                    te = j;
                } else {
                    L[j][j] = sqrt(d);
#pragma unroll
                    for (int i = j + 1; i < T; ++i) {
                        if (i < te) {
                            double v = L[i][j];
#pragma unroll
                            for (int k = 0; k < j; ++k) v = __fma_rn(-L[i][k], L[j][k], v);
                            L[i][j] = v / L[j][j];
                        }
                    }
                }
            }
        }
    }
    if (te == 1) {
        alpha[0] = phi[1] / phi[2];
        return 1;
    }
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if (i < te) {
            double v = g[i];
#pragma unroll
            for (int k = 0; k < i; ++k) v = __fma_rn(-L[i][k], z[k], v);
            z[i] = v / L[i][i];
        }
    }
#pragma unroll
    for (int i = T - 1; i >= 0; --i) {
        if (i < te) {
            double v = z[i];
#pragma unroll
            for (int k = i + 1; k < T; ++k)
                if (k < te) v = __fma_rn(-L[k][i], at[k], v);
            at[i] = v / L[i][i];
        }
    }
#pragma unroll
    for (int i = 0; i < T; ++i)
        if (i < te) alpha[i] = s[i] * at[i];
    return te;
}

__device__ inline int gram_alpha(const double *phi, int t, double *alpha) {
    switch (t) {
        case 1: return gram_alpha_t<1>(phi, alpha);
        case 2: return gram_alpha_t<2>(phi, alpha);
        case 3: return gram_alpha_t<3>(phi, alpha);
        case 4: return gram_alpha_t<4>(phi, alpha);
        case 5: return gram_alpha_t<5>(phi, alpha);
        case 6: return gram_alpha_t<6>(phi, alpha);
        case 7: return gram_alpha_t<7>(phi, alpha);
        default: return gram_alpha_t<8>(phi, alpha);
    }
}

}  // namespace ta
