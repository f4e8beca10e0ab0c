// The per-node adjoint update shared by the adjoint kernels (lbm_adjoint.hip) and the
// multi-level adjoint kernel (lbm_march_adj.hip), and the probe source of a node.  Both
// take every node's arithmetic from here, which is what makes the fused levels bit for bit
// the single steps.  The adjoint of one level at one node, mirroring the forward step:
//   g = dL/dU^m = omega sum_q (f^eq_q)'(U^m)^T lambda*^m_q
//   lambda^m_q = (1 - omega) lambda*^m_q + g
// with (f^eq_q)' from eq:feq-derivative and the Jacobian actions of eq:jacobian-actions
// through the tangent C = dP/dF (eq:stress-and-tangent), used transposed.
#pragma once

#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"

namespace lbm {

// One node of the adjoint step (see above): the pulled lambda*^m l and the state F - I of
// the record -> lambda^m (out) and the increments of this level's parameter gradients
// (inc: mu, lam, b1, b2; zero where not asked for).
template <typename R, int LAW>
__device__ __forceinline__ void adj_node(const Common& cm, const R l[4][6], const R ft[4], R mu, R lam, R rm,
                                         bool grad_par, bool grad_body, R out[4][6], R inc[4]) {
    // log-NH and NH: one evaluation of the kinematics gives the tangent's action and, below,
    // dP/dmu = F - H and dP/dlam = ln J H (log-NH) or (J^2 - 1)/2 H (NH)
    constexpr bool lame = LAW == LBM_LOGNH || LAW == LBM_NH;
    R s6[6], dxl[6], dyl[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        s6[k] = l[0][k] + l[1][k] + l[2][k] + l[3][k];
        dxl[k] = l[0][k] - l[2][k];
        dyl[k] = l[1][k] - l[3][k];
    }
    // AT_kB = -sum_iA W_iA C_iAkB with W = [[dxl0, dyl0], [dxl1, dyl1]] (the flux rows that
    // carry P_i1 and P_i2)
    R AT[6];
    AT[0] = -dxl[2] - dyl[3];
    AT[1] = -dxl[4] - dyl[5];
    Kin<R> kk;
    if constexpr (lame) {
        // with C_iAkB = mu d_ik d_AB + a H_iB H_kA + b H_iA H_kB (tangent_lame) the action
        // needs no C: AT_kB = -(mu W_kB + a (H M^T)_kB + b tr(M) H_kB), M = H^T W
        kk = kinematics<R, true>(ft);
        R a, b;
        if constexpr (LAW == LBM_LOGNH) {
            a = mu - lam * kk.L;
            b = lam;
        } else {
            a = mu - R(0.5) * lam * kk.Jsq_m1;
            b = lam * kk.J * kk.J;
        }
        const R* H = kk.H;
        const R W[2][2] = {{dxl[0], dyl[0]}, {dxl[1], dyl[1]}};
        R M[2][2];
#pragma unroll
        for (int B = 0; B < 2; ++B)
#pragma unroll
            for (int A = 0; A < 2; ++A) M[B][A] = H[B] * W[0][A] + H[2 + B] * W[1][A];
        const R tr = M[0][0] + M[1][1];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int B = 0; B < 2; ++B) {
                const R hm = H[2 * k] * M[B][0] + H[2 * k + 1] * M[B][1];
                AT[2 + 2 * k + B] = -(mu * W[k][B] + a * hm + b * tr * H[2 * k + B]);
            }
    } else {
        R C[16];
        tangent<R, LAW, true>(ft, mu, lam, law_consts<R>(cm), C);
#pragma unroll
        for (int kB = 0; kB < 4; ++kB)
            AT[2 + kB] = -(dxl[0] * C[kB] + dxl[1] * C[8 + kB]) - (dyl[0] * C[4 + kB] + dyl[1] * C[12 + kB]);
    }
    const R om = kval<R>(cm.omega, cm.f_omega);
    const R c2 = kval<R>(cm.k_c2, cm.f_c2);
    R gU[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gU[k] = om * R(0.25) * (s6[k] + c2 * AT[k]);
    const R omc = R(1) - om;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) out[q][k] = omc * l[q][k] + gU[k];
    const R hc = kval<R>(cm.k_hc, cm.f_hc);
    inc[0] = inc[1] = inc[2] = inc[3] = R(0);
    if (grad_par) {
        R Pm[4], Pl[4];
        if constexpr (lame) {
            const R v = LAW == LBM_LOGNH ? kk.L : R(0.5) * kk.Jsq_m1;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                Pm[a] = kk.FmH[a];
                Pl[a] = v * kk.H[a];
            }
        } else {
            piola_partials<R, LAW, true>(ft, law_consts<R>(cm), Pm, Pl);
        }
        inc[0] = om * hc * -(dxl[0] * Pm[0] + dxl[1] * Pm[2] + dyl[0] * Pm[1] + dyl[1] * Pm[3]);
        inc[1] = om * hc * -(dxl[0] * Pl[0] + dxl[1] * Pl[2] + dyl[0] * Pl[1] + dyl[1] * Pl[3]);
    }
    if (grad_body) {
        const R hdtr = kval<R>(cm.k_hdt, cm.f_hdt), srcw = kval<R>(cm.k_srcw, cm.f_srcw);
        inc[2] = rm * (hdtr * gU[0] + srcw * s6[0]);
        inc[3] = rm * (hdtr * gU[1] + srcw * s6[1]);
    }
}

// Probe source of the level at node (x, y) if it is a probe (bit x mod 64 of the word of
// its tile row in the probe table): lambda_q += weight ubar for every q (the sum of the
// ubar of every probe on that cell).  Without a table the probes are walked by
// adj_probe_kernel instead.
template <typename R, typename Args>
__device__ __forceinline__ bool probe_at(const Args& a, int x, int y, double src[2]) {
    if (!a.pmask) return false;
    const uint64_t word = a.pmask[int64_t(y) * a.cm.ntile + (x >> 6)];
    if (!((word >> (x & 63)) & 1ull)) return false;
    const int64_t n = int64_t(a.cm.nx) * a.cm.ny, idx = int64_t(y) * a.cm.nx + x;
    src[0] = a.probe_weight * a.pfield[idx];
    src[1] = a.probe_weight * a.pfield[n + idx];
    return true;
}

}  // namespace lbm
