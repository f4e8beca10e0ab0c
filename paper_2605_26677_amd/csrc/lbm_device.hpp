// Device building blocks of the D2Q4 x 6 vectorial LBM: storage traits, the hyperelastic
// closures of the paper's Appendix A evaluated in registers, their tangents
// (eq:stress-and-tangent), and small helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// ---------------------------------------------------------------- storage traits

template <int ST> struct Storage;
template <> struct Storage<LBM_F32_SHIFTED> {
    using pop_t = float;
    using real = float;
    static constexpr bool shifted = true;
};
template <> struct Storage<LBM_F16_SHIFTED> {
    using pop_t = _Float16;
    using real = float;
    static constexpr bool shifted = true;
};
template <> struct Storage<LBM_F64_PLAIN> {
    using pop_t = double;
    using real = double;
    static constexpr bool shifted = false;
};

template <typename T, typename R> __device__ __forceinline__ R load_as(const T* p) {
    return static_cast<R>(*p);
}
// float -> _Float16 conversion is round-to-nearest-even with subnormals kept.
template <typename T, typename R> __device__ __forceinline__ void store_as(T* p, R v) {
    *p = static_cast<T>(v);
}

// 2 atanh(s) = ln((1 + s) / (1 - s)) for |s| <= 1/5 by its Taylor series
// 2 (s + s^3/3 + ... + s^11/11): the first omitted term is below 2^-27 of the sum.
__device__ __forceinline__ float atanh2_series(float s) {
    const float s2 = s * s;
    float t = 1.0f / 11.0f;
    t = fmaf(t, s2, 1.0f / 9.0f);
    t = fmaf(t, s2, 1.0f / 7.0f);
    t = fmaf(t, s2, 1.0f / 5.0f);
    t = fmaf(t, s2, 1.0f / 3.0f);
    const float d = 2.0f * s;
    return fmaf(d * s2, t, d);
}

// ln(1 + x) in FP32 from ln(1 + x) = 2 atanh(x / (2 + x)).  For -1/4 <= x < 1/2 (|J - 1| of
// every state the workloads reach) the series applies directly, so a small x keeps its
// relative accuracy; elsewhere 1 + x = m 2^e with m in [sqrt(1/2), sqrt(2)) and
// ln(1 + x) = e ln 2 + 2 atanh((m - 1) / (m + 1)).  The quotients use the hardware
// reciprocal; the result is within a few units in the last place (checked against FP64
// through lbm_stress), at about a tenth of the instructions of the library's log1pf, whose
// compensated arithmetic the collision does not need.
__device__ __forceinline__ float log1p_r(float x) {
    if (x >= -0.25f && x < 0.5f) return atanh2_series(x * __builtin_amdgcn_rcpf(2.0f + x));
    const float u = 1.0f + x;
    if (!(u > 0.0f)) return u == 0.0f ? -__builtin_inff() : __builtin_nanf("");
    if (u == __builtin_inff()) return u;
    int e;
    float m = frexpf(u, &e);                  // u = m 2^e, m in [1/2, 1)
    if (m < 0.70710678f) {
        m *= 2.0f;
        e -= 1;
    }
    return fmaf(float(e), 0.69314718f, atanh2_series((m - 1.0f) * __builtin_amdgcn_rcpf(m + 1.0f)));
}
__device__ __forceinline__ double log1p_r(double x) { return log1p(x); }
__device__ __forceinline__ float expm1_r(float x) { return expm1f(x); }
__device__ __forceinline__ double expm1_r(double x) { return expm1(x); }
__device__ __forceinline__ float log_r(float x) { return logf(x); }
__device__ __forceinline__ double log_r(double x) { return log(x); }
__device__ __forceinline__ float sqrt_r(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
__device__ __forceinline__ bool finite_r(float x) { return isfinite(x); }
__device__ __forceinline__ bool finite_r(double x) { return isfinite(x); }

// D2Q4 directions in the paper's order (Sec. 3.1).
__host__ __device__ constexpr int dir_i(int q) { return q == 0 ? 1 : (q == 2 ? -1 : 0); }
__host__ __device__ constexpr int dir_j(int q) { return q == 1 ? 1 : (q == 3 ? -1 : 0); }

// ---------------------------------------------------------------- kinematics
//
// A deformation state is passed as four numbers f[0..3] = (11, 12, 21, 22): the shift
// F - I when SHIFTED, the plain F otherwise.  With the shift, J - 1 and F - F^{-T} are
// formed without subtracting nearly equal numbers:
//   delta = J - 1 = f11 + f22 + (f11 f22 - f12 f21),
//   F - H = (1/J) [[f11 - f22 + delta (1 + f11), J f12 + f21],
//                  [J f21 + f12, f22 - f11 + delta (1 + f22)]],   H = F^{-T}.

// 1/x: the hardware reciprocal in FP32 (within 1 ulp), the correctly rounded quotient in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename R> struct Kin {
    R J, invJ, L;          // det F, 1/J, ln J
    R H[4];                // F^{-T}
    R FmH[4];              // F - F^{-T}
    R Jsq_m1;              // J^2 - 1
};

template <typename R, bool SHIFTED>
__device__ __forceinline__ Kin<R> kinematics(const R f[4]) {
    Kin<R> k;
    if constexpr (SHIFTED) {
        const R d = f[0] + f[3] + (f[0] * f[3] - f[1] * f[2]);
        k.J = R(1) + d;
        k.invJ = recip(k.J);
        k.L = log1p_r(d);
        k.Jsq_m1 = d * (R(2) + d);
        k.H[0] = (R(1) + f[3]) * k.invJ;
        k.H[1] = -f[2] * k.invJ;
        k.H[2] = -f[1] * k.invJ;
        k.H[3] = (R(1) + f[0]) * k.invJ;
        k.FmH[0] = (f[0] - f[3] + d * (R(1) + f[0])) * k.invJ;
        k.FmH[1] = (k.J * f[1] + f[2]) * k.invJ;
        k.FmH[2] = (k.J * f[2] + f[1]) * k.invJ;
        k.FmH[3] = (f[3] - f[0] + d * (R(1) + f[3])) * k.invJ;
    } else {
        k.J = f[0] * f[3] - f[1] * f[2];
        k.invJ = recip(k.J);
        k.L = log_r(k.J);
        k.Jsq_m1 = k.J * k.J - R(1);
        k.H[0] = f[3] * k.invJ;
        k.H[1] = -f[2] * k.invJ;
        k.H[2] = -f[1] * k.invJ;
        k.H[3] = f[0] * k.invJ;
        for (int a = 0; a < 4; ++a) k.FmH[a] = f[a] - k.H[a];
    }
    return k;
}

template <typename R, bool SHIFTED>
__device__ __forceinline__ void full_F(const R f[4], R F[4]) {
    if constexpr (SHIFTED) {
        F[0] = R(1) + f[0]; F[1] = f[1]; F[2] = f[2]; F[3] = R(1) + f[3];
    } else {
        F[0] = f[0]; F[1] = f[1]; F[2] = f[2]; F[3] = f[3];
    }
}

// Green-Lagrange strain E = (F^T F - I)/2 as (E11, E12, E22); from the shift
// E = (F~ + F~^T + F~^T F~)/2.
template <typename R, bool SHIFTED>
__device__ __forceinline__ void green_lagrange(const R f[4], R& E11, R& E12, R& E22) {
    if constexpr (SHIFTED) {
        E11 = f[0] + R(0.5) * (f[0] * f[0] + f[2] * f[2]);
        E22 = f[3] + R(0.5) * (f[1] * f[1] + f[3] * f[3]);
        E12 = R(0.5) * (f[1] + f[2] + f[0] * f[1] + f[2] * f[3]);
    } else {
        E11 = R(0.5) * (f[0] * f[0] + f[2] * f[2] - R(1));
        E22 = R(0.5) * (f[1] * f[1] + f[3] * f[3] - R(1));
        E12 = R(0.5) * (f[0] * f[1] + f[2] * f[3]);
    }
}

// ---------------------------------------------------------------- law constants
// Constants of the invariant-based closures as multiples of mu (P stays linear in mu and
// lam): Mooney-Rivlin (k0, k1) = (c10, c01)/mu; Yeoh (k0, k1, k2) = (c1, c2, c3)/mu;
// Gent k0 = J_m.  Unused by the Lame-parametrised laws.
template <typename R> struct LawK {
    R k0, k1, k2;
};

// ---------------------------------------------------------------- forward-mode duals
// A value with its derivatives along four seed directions; used to differentiate the
// invariant-based stresses (one pass gives all 16 tangent entries).
template <typename R> struct Dual4 {
    R v;
    R d[4];
};
template <typename R> __device__ __forceinline__ Dual4<R> operator+(const Dual4<R>& a, const Dual4<R>& b) {
    Dual4<R> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator+(const Dual4<R>& a, R b) {
    Dual4<R> r = a;
    r.v = a.v + b;
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator+(R a, const Dual4<R>& b) { return b + a; }
template <typename R> __device__ __forceinline__ Dual4<R> operator-(const Dual4<R>& a) {
    Dual4<R> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = -a.d[i];
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator-(const Dual4<R>& a, const Dual4<R>& b) {
    Dual4<R> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator-(const Dual4<R>& a, R b) {
    Dual4<R> r = a;
    r.v = a.v - b;
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator-(R a, const Dual4<R>& b) {
    Dual4<R> r = -b;
    r.v = a - b.v;
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator*(const Dual4<R>& a, const Dual4<R>& b) {
    Dual4<R> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator*(const Dual4<R>& a, R b) {
    Dual4<R> r;
    r.v = a.v * b;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator*(R a, const Dual4<R>& b) { return b * a; }
template <typename R> __device__ __forceinline__ Dual4<R> operator/(const Dual4<R>& a, const Dual4<R>& b) {
    const R inv = R(1) / b.v;
    Dual4<R> r;
    r.v = a.v * inv;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> operator/(R a, const Dual4<R>& b) {
    const R inv = R(1) / b.v;
    Dual4<R> r;
    r.v = a * inv;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = -r.v * b.d[i] * inv;
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> log1p_r(const Dual4<R>& a) {
    const R s = R(1) / (R(1) + a.v);
    Dual4<R> r;
    r.v = log1p_r(a.v);
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] * s;
    return r;
}
template <typename R> __device__ __forceinline__ Dual4<R> expm1_r(const Dual4<R>& a) {
    Dual4<R> r;
    r.v = expm1_r(a.v);
    const R s = r.v + R(1);
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] * s;
    return r;
}

// ---------------------------------------------------------------- invariant-based closures
// Mooney-Rivlin, Yeoh and Gent (eq:mr-model, eq:yeoh-model, eq:gent-model) on the shift
// f = F - I, for a scalar S that is R or Dual4<R>.  With t = tr C - 2 = I1 - 3,
// s = J^2 - 1 = delta (2 + delta), L = ln J = log1p(delta) and j = J^{-2/3} = 1 + expm1(-2L/3),
// the invariant gradients of eq:modified-invariant-gradients become
//   G1 = j [2 (F - H) - (2/3) t H],
//   G2 = j^2 [2 (F - H) + ((2/3) s - (4/3) t) H],
// and A = barI1 - 3 = j t + 3 expm1(-2L/3): every term vanishes at F = I on its own, so
// small strains do not cancel against O(1) quantities.  Outputs P and (J, A) for the
// admissibility checks (J > 0; Gent also A < J_m).
template <typename S, typename R, int LAW>
__device__ __forceinline__ void piola_invariant(const S f[4], R mu, R lam, const LawK<R>& lk, S P[4],
                                                S& J, S& A) {
    const S d = f[0] + f[3] + (f[0] * f[3] - f[1] * f[2]);
    J = R(1) + d;
    const S invJ = R(1) / J;
    const S L = log1p_r(d);
    const S H[4] = {(R(1) + f[3]) * invJ, -(f[2] * invJ), -(f[1] * invJ), (R(1) + f[0]) * invJ};
    const S FmH[4] = {(f[0] - f[3] + d * (R(1) + f[0])) * invJ, (J * f[1] + f[2]) * invJ,
                      (J * f[2] + f[1]) * invJ, (f[3] - f[0] + d * (R(1) + f[3])) * invJ};
    const S t = R(2) * (f[0] + f[3]) + (f[0] * f[0] + f[1] * f[1] + f[2] * f[2] + f[3] * f[3]);
    const S em = expm1_r(R(-2.0 / 3.0) * L);
    const S j = R(1) + em;
    A = j * t + R(3) * em;
    const S volL = lam * L;
    if constexpr (LAW == LBM_MR) {
        const S sJ = d * (R(2) + d);
        const S a1 = (mu * lk.k0) * j;
        const S a2 = (mu * lk.k1) * (j * j);
        const S h1 = R(-2.0 / 3.0) * t;
        const S h2 = R(2.0 / 3.0) * sJ + R(-4.0 / 3.0) * t;
#pragma unroll
        for (int a = 0; a < 4; ++a)
            P[a] = a1 * (R(2) * FmH[a] + h1 * H[a]) + a2 * (R(2) * FmH[a] + h2 * H[a]) + volL * H[a];
    } else {
        S alpha;
        if constexpr (LAW == LBM_YEOH) alpha = mu * (lk.k0 + A * (R(2) * lk.k1 + R(3) * lk.k2 * A));
        else alpha = (R(0.5) * mu) / (R(1) - A * (R(1) / lk.k0));
        const S aj = alpha * j;
        const S h1 = R(-2.0 / 3.0) * t;
#pragma unroll
        for (int a = 0; a < 4; ++a) P[a] = aj * (R(2) * FmH[a] + h1 * H[a]) + volL * H[a];
    }
}

template <int LAW> constexpr bool invariant_law() {
    return LAW == LBM_MR || LAW == LBM_YEOH || LAW == LBM_GENT;
}

// Shifted copy of a plain or shifted deformation state.
template <typename R, bool SHIFTED>
__device__ __forceinline__ void to_shift(const R f[4], R fs[4]) {
    fs[0] = SHIFTED ? f[0] : f[0] - R(1);
    fs[1] = f[1];
    fs[2] = f[2];
    fs[3] = SHIFTED ? f[3] : f[3] - R(1);
}

// ---------------------------------------------------------------- first Piola stress
// P(F) of Appendix A in registers; also returns J for the admissibility check (J is
// reported as 0 for a Gent state beyond the limit A < J_m, so that every caller's J > 0
// test also rejects it).

template <typename R, int LAW, bool SHIFTED>
__device__ __forceinline__ void piola(const R f[4], R mu, R lam, const LawK<R>& lk, R P[4], R& J) {
    if constexpr (invariant_law<LAW>()) {
        R fs[4], A;
        to_shift<R, SHIFTED>(f, fs);
        piola_invariant<R, R, LAW>(fs, mu, lam, lk, P, J, A);
        if (LAW == LBM_GENT && !(A < lk.k0)) J = R(0);
    } else if constexpr (LAW == LBM_SVK) {
        R E11, E12, E22;
        green_lagrange<R, SHIFTED>(f, E11, E12, E22);
        const R tr = E11 + E22;
        const R S11 = R(2) * mu * E11 + lam * tr, S22 = R(2) * mu * E22 + lam * tr;
        const R S12 = R(2) * mu * E12;
        R F[4];
        full_F<R, SHIFTED>(f, F);
        P[0] = F[0] * S11 + F[1] * S12;
        P[1] = F[0] * S12 + F[1] * S22;
        P[2] = F[2] * S11 + F[3] * S12;
        P[3] = F[2] * S12 + F[3] * S22;
        if constexpr (SHIFTED) J = R(1) + (f[0] + f[3] + (f[0] * f[3] - f[1] * f[2]));
        else J = f[0] * f[3] - f[1] * f[2];
    } else {
        const Kin<R> k = kinematics<R, SHIFTED>(f);
        const R vol = (LAW == LBM_LOGNH) ? lam * k.L : R(0.5) * lam * k.Jsq_m1;
        for (int a = 0; a < 4; ++a) P[a] = mu * k.FmH[a] + vol * k.H[a];
        J = k.J;
    }
}

// dP/dmu and dP/dlam (every law here is linear in the two parameters).
template <typename R, int LAW, bool SHIFTED>
__device__ __forceinline__ void piola_partials(const R f[4], const LawK<R>& lk, R Pm[4], R Pl[4]) {
    R J;
    piola<R, LAW, SHIFTED>(f, R(1), R(0), lk, Pm, J);
    piola<R, LAW, SHIFTED>(f, R(0), R(1), lk, Pl, J);
}

// ---------------------------------------------------------------- tangent
// C[i][A][k][B] = dP_iA / dF_kB stored at index 8 i + 4 A + 2 k + B.  The closed forms
// follow by differentiating Appendix A (H = F^{-T}, L = ln J, S = lam tr E I + 2 mu E):
//   log-NH: mu d_ik d_AB + (mu - lam L) H_iB H_kA + lam H_iA H_kB
//   NH:     mu d_ik d_AB + (mu - lam (J^2 - 1)/2) H_iB H_kA + lam J^2 H_iA H_kB
//   SVK:    d_ik S_AB + lam F_iA F_kB + mu (F_iB F_kA + (F F^T)_ik d_AB)
// The invariant-based laws are differentiated in forward mode (Dual4 seeded with the four
// entries of F), which is exact up to rounding like the closed forms.

// The tangent of log-NH and NH from the kinematics of the state.
template <typename R, int LAW>
__device__ __forceinline__ void tangent_lame(const Kin<R>& kk, R mu, R lam, R C[16]) {
    R a, b;
    if constexpr (LAW == LBM_LOGNH) {
        a = mu - lam * kk.L;
        b = lam;
    } else {
        a = mu - R(0.5) * lam * kk.Jsq_m1;
        b = lam * kk.J * kk.J;
    }
    const R* H = kk.H;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int B = 0; B < 2; ++B) {
                    R v = a * H[2 * i + B] * H[2 * k + A] + b * H[2 * i + A] * H[2 * k + B];
                    if (i == k && A == B) v += mu;
                    C[8 * i + 4 * A + 2 * k + B] = v;
                }
}

template <typename R, int LAW, bool SHIFTED>
__device__ __forceinline__ void tangent(const R f[4], R mu, R lam, const LawK<R>& lk, R C[16]) {
    if constexpr (invariant_law<LAW>()) {
        R fs[4];
        to_shift<R, SHIFTED>(f, fs);
        Dual4<R> fd[4], P[4], J, A;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            fd[a].v = fs[a];
#pragma unroll
            for (int b = 0; b < 4; ++b) fd[a].d[b] = (a == b) ? R(1) : R(0);
        }
        piola_invariant<Dual4<R>, R, LAW>(fd, mu, lam, lk, P, J, A);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) C[4 * a + b] = P[a].d[b];
    } else if constexpr (LAW == LBM_SVK) {
        R E11, E12, E22;
        green_lagrange<R, SHIFTED>(f, E11, E12, E22);
        const R tr = E11 + E22;
        const R S[4] = {R(2) * mu * E11 + lam * tr, R(2) * mu * E12, R(2) * mu * E12,
                        R(2) * mu * E22 + lam * tr};
        R F[4];
        full_F<R, SHIFTED>(f, F);
        R FFt[4];
        FFt[0] = F[0] * F[0] + F[1] * F[1];
        FFt[1] = F[0] * F[2] + F[1] * F[3];
        FFt[2] = FFt[1];
        FFt[3] = F[2] * F[2] + F[3] * F[3];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int A = 0; A < 2; ++A)
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int B = 0; B < 2; ++B) {
                        R v = lam * F[2 * i + A] * F[2 * k + B] + mu * F[2 * i + B] * F[2 * k + A];
                        if (i == k) v += S[2 * A + B];
                        if (A == B) v += mu * FFt[2 * i + k];
                        C[8 * i + 4 * A + 2 * k + B] = v;
                    }
    } else {
        tangent_lame<R, LAW>(kinematics<R, SHIFTED>(f), mu, lam, C);
    }
}

// Strain energy W(F) (Appendix A), used by the diagnostics.
template <typename R, int LAW, bool SHIFTED>
__device__ __forceinline__ R energy(const R f[4], R mu, R lam, const LawK<R>& lk) {
    if constexpr (invariant_law<LAW>()) {
        R fs[4];
        to_shift<R, SHIFTED>(f, fs);
        const R d = fs[0] + fs[3] + (fs[0] * fs[3] - fs[1] * fs[2]);
        const R L = log1p_r(d);
        const R t = R(2) * (fs[0] + fs[3]) + (fs[0] * fs[0] + fs[1] * fs[1] + fs[2] * fs[2] + fs[3] * fs[3]);
        const R em = expm1_r(R(-2.0 / 3.0) * L);
        const R A = (R(1) + em) * t + R(3) * em;
        const R vol = R(0.5) * lam * L * L;
        if constexpr (LAW == LBM_MR) {
            // barI2 - 3 = J^{-4/3} (s + t) + 3 expm1(-4L/3), s = J^2 - 1
            const R em4 = expm1_r(R(-4.0 / 3.0) * L);
            const R A2 = (R(1) + em4) * (d * (R(2) + d) + t) + R(3) * em4;
            return mu * (lk.k0 * A + lk.k1 * A2) + vol;
        } else if constexpr (LAW == LBM_YEOH) {
            return mu * A * (lk.k0 + A * (lk.k1 + A * lk.k2)) + vol;
        } else {
            return R(-0.5) * mu * lk.k0 * log1p_r(-A / lk.k0) + vol;
        }
    } else if constexpr (LAW == LBM_SVK) {
        R E11, E12, E22;
        green_lagrange<R, SHIFTED>(f, E11, E12, E22);
        const R tr = E11 + E22;
        return R(0.5) * lam * tr * tr + mu * (E11 * E11 + R(2) * E12 * E12 + E22 * E22);
    } else {
        const Kin<R> k = kinematics<R, SHIFTED>(f);
        // tr C - 2 - 2 ln J, with tr C - 2 = 2 (f11 + f22) + |f|^2 in shifted form
        R trCm2;
        if constexpr (SHIFTED)
            trCm2 = R(2) * (f[0] + f[3]) + f[0] * f[0] + f[1] * f[1] + f[2] * f[2] + f[3] * f[3];
        else
            trCm2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2] + f[3] * f[3] - R(2);
        const R dev = R(0.5) * mu * (trCm2 - R(2) * k.L);
        if constexpr (LAW == LBM_LOGNH) return dev + R(0.5) * lam * k.L * k.L;
        else return dev + R(0.25) * lam * (k.Jsq_m1 - R(2) * k.L);
    }
}

// ---------------------------------------------------------------- tiled layout
//
// Arrays of per-node planes (populations: 24, u*: 4 or 2, records: 6) are stored in
// tiles of kTile consecutive nodes of one row; a tile holds all its planes contiguously:
// element (p, x, y) of an np-plane array sits at ((y * ntile + x / kTile) * np + p) * kTile
// + x mod kTile, ntile = ceil(nx / kTile).  One wavefront of 64 lanes covers one tile, so
// a pass over the grid reads and writes a few long contiguous runs per wavefront instead
// of one short run in each of 24 + 24 + 4 + 4 widely separated planes.

constexpr int kTile = 64;

__host__ __device__ __forceinline__ int64_t tile_base(int ntile, int np, int x, int y) {
    return ((int64_t(y) * ntile + (x >> 6)) * np) * kTile + (x & (kTile - 1));
}

// Displacement accumulator of the shifted storages (F32, F16): u* = U + S, with S two
// tiled float planes that collect dt v over at most kUstarBlock steps and U two tiled
// double planes (after the S planes) that receive S at the steps n -> n+1 with
// (n + 1) % kUstarBlock == 0.  S restarts from zero every block, so its rounding stays on
// the scale of one block's increment while U keeps the sum exact to FP64; a step moves
// 16 bytes per node instead of the 32 of a compensated float pair.
constexpr int kUstarBlock = 16;
// Levels per FP32 block sum of the adjoint's parameter gradients (same scheme: the FP64
// gradient receives a block sum every kGradBlock levels).
constexpr int kGradBlock = 16;

struct UstarRefs {
    float* S;
    double* U;
};
__host__ __device__ __forceinline__ UstarRefs ustar_refs(void* base, int ntile, int ny, int x, int y) {
    const int64_t padded = int64_t(ntile) * kTile * ny;
    UstarRefs r;
    r.S = (float*)base + tile_base(ntile, 2, x, y);
    r.U = (double*)((float*)base + 2 * padded) + tile_base(ntile, 2, x, y);
    return r;
}

// Store that bypasses the caches' allocate-on-write (each value is written once per pass).
// A computed value rounded to the population storage type: the compute-type result is
// formed first and then rounded to nearest even.  The empty asm keeps the compiler from
// fusing the rounding into the instruction that produced the value (a mixed-precision FMA
// rounds once, straight to half), so every kernel rounds a population the same way.
template <typename T, typename R> __device__ __forceinline__ T to_storage(R v) {
    if constexpr (sizeof(T) == sizeof(R)) {
        return v;
    } else {
        asm("" : "+v"(v));
        return T(v);
    }
}

template <typename T> __device__ __forceinline__ void store_stream(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Second-order first derivative of g along an axis of length L at position s: central
// differences, periodic wrap, or the one-sided three-point formula at the ends of a
// non-periodic axis.  get(s') returns the value at s'.
template <typename R, typename Get>
__device__ __forceinline__ R fd_along(Get get, int s, int L, bool periodic, R inv2h) {
    if (periodic) {
        const int sp = (s + 1 == L) ? 0 : s + 1;
        const int sm = (s == 0) ? L - 1 : s - 1;
        return (get(sp) - get(sm)) * inv2h;
    }
    if (s == 0) return (R(-3) * get(0) + R(4) * get(1) - get(2)) * inv2h;
    if (s == L - 1) return (R(3) * get(L - 1) - R(4) * get(L - 2) + get(L - 3)) * inv2h;
    return (get(s + 1) - get(s - 1)) * inv2h;
}

// Column s of the same difference operator, applied as a transpose:
// sum over rows s' of D[s', s] * gbar(s').
template <typename R, typename Get>
__device__ __forceinline__ R fd_along_T(Get gbar, int s, int L, bool periodic, R inv2h) {
    if (periodic) {
        const int sp = (s + 1 == L) ? 0 : s + 1;
        const int sm = (s == 0) ? L - 1 : s - 1;
        return (gbar(sm) - gbar(sp)) * inv2h;
    }
    R acc = R(0);
    // central rows s' in [1, L-2]: D[s', s'+1] = +1, D[s', s'-1] = -1
    if (s - 1 >= 1 && s - 1 <= L - 2) acc += gbar(s - 1);
    if (s + 1 >= 1 && s + 1 <= L - 2) acc -= gbar(s + 1);
    // row 0: (-3, 4, -1) on columns 0, 1, 2
    if (s == 0) acc += R(-3) * gbar(0);
    if (s == 1) acc += R(4) * gbar(0);
    if (s == 2) acc += R(-1) * gbar(0);
    // row L-1: (1, -4, 3) on columns L-3, L-2, L-1
    if (s == L - 1) acc += R(3) * gbar(L - 1);
    if (s == L - 2) acc += R(-4) * gbar(L - 1);
    if (s == L - 3) acc += R(1) * gbar(L - 1);
    return acc * inv2h;
}

// Per-edge geometry (Sec. 3.6): outward normal, axis A the normal is aligned with,
// missing incoming direction d = -N and its opposite.
struct EdgeGeom {
    int A;        // 0 for x-edges (normal along X), 1 for y-edges
    int NA;       // normal component along A (+1 or -1)
    int d;        // missing incoming direction at the wall nodes
    int od;       // outgoing direction -d = N
};
__host__ __device__ constexpr EdgeGeom edge_geom(int e) {
    return e == LBM_XMIN ? EdgeGeom{0, -1, 0, 2}
         : e == LBM_XMAX ? EdgeGeom{0, 1, 2, 0}
         : e == LBM_YMIN ? EdgeGeom{1, -1, 1, 3}
                         : EdgeGeom{1, 1, 3, 1};
}

}  // namespace lbm
