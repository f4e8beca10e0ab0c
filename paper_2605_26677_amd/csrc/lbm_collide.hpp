// The per-node update shared by the single-step kernel (lbm_forward.hip) and the two-level
// kernels (lbm_pair.hip): the wall links, the collision and the state record.  Both files
// take every node's arithmetic from here, which is what makes two fused levels bit for
// bit two single steps.
#pragma once

#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"

namespace lbm {
// Missing link d at a wall node of edge e (eq:boundary-general):
// f_d = D f*_{-d}(X) + S_d, velocity rule eq:dirichlet-boundary-rule,
// traction rule eq:neumann-boundary-rule.  In shifted storage only the traction F rows
// change: g_d = -g*_{-d} + (F^b - I)/2 (F^b arrives from the staging buffer as F^b - I).
// ownp points at the node's first population, plane stride `stride` (the tiled array or a
// wall line of the staging buffer).
template <typename T, typename R>
__device__ __forceinline__ void wall_link(const Common& cm, const EdgeData& ed, const void* auxp,
                                          int e, int s, const T* ownp, int64_t stride, R out[6]) {
    const EdgeGeom G = edge_geom(e);
    const int L = (G.A == 0) ? cm.ny : cm.nx;
    R o[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = R(ownp[(6 * G.od + k) * stride]);
    const R w0 = edge_value<R>(ed, e, 0, s, L), w1 = edge_value<R>(ed, e, 1, s, L);
    const R c = R(cm.c);
    if (cm.bc[e] == LBM_VELOCITY) {
        const R N0 = (G.A == 0) ? R(G.NA) : R(0), N1 = (G.A == 1) ? R(G.NA) : R(0);
        out[0] = -o[0] + R(0.5) * w0;
        out[1] = -o[1] + R(0.5) * w1;
        out[2] = o[2] + N0 * w0 / c;
        out[3] = o[3] + N1 * w0 / c;
        out[4] = o[4] + N0 * w1 / c;
        out[5] = o[5] + N1 * w1 / c;
    } else {
        int off[4], len[4];
        edge_offsets(cm.nx, cm.ny, off, len);
        const R* Fb = (const R*)auxp + 4 * (int64_t)(off[e] + s);
        out[0] = o[0] + w0 / c;
        out[1] = o[1] + w1 / c;
#pragma unroll
        for (int k = 0; k < 4; ++k) out[2 + k] = -o[2 + k] + R(0.5) * Fb[k];
    }
}

// One node's update from its pulled populations g: moments with the half-step source
// (eq:moment-U), the constitutive response in registers, fluxes (eq:flux-vectors),
// equilibrium (eq:feq) and the collision with trapezoidal forcing (eq:collision).
// B0, B1: body acceleration at the new level.  Returns the post-collision populations
// and U (velocity rows include the half-step source).
template <typename R, int LAW, bool SH>
__device__ __forceinline__ void collide_node(const Common& cm, const R g[4][6], R B0, R B1, R mu, R lam,
                                             R out[4][6], R U[6], R& J) {
    const R hdt = kval<R>(cm.k_hdt, cm.f_hdt);
#pragma unroll
    for (int k = 0; k < 6; ++k) U[k] = g[0][k] + g[1][k] + g[2][k] + g[3][k];
    U[0] += hdt * B0;
    U[1] += hdt * B1;
    R P[4];
    piola<R, LAW, SH>(&U[2], mu, lam, law_consts<R>(cm), P, J);
    // f*_q = (1 - omega) f_q + omega f^eq_q + source, with
    // omega f^eq_q = (omega/4) U + (omega/(2c)) (i Phi_X + j Phi_Y) for e_q = (i, j) and the
    // fluxes Phi_X = -(P11, P21, v1, 0, v2, 0), Phi_Y = -(P12, P22, 0, v1, 0, v2)
    // (eq:flux-vectors); the zero entries and the unit factors i, j are taken out by hand.
    // omc = 1 - 4 omq is exact in R (Sterbenz), so the weights of f and f^eq sum to exactly
    // 1 and the collision keeps sum_q f* = U + (dt/2) B without a drift of the moments
    const R omq = kval<R>(cm.k_omq, cm.f_omq), omc = R(1) - R(4) * omq, cq = kval<R>(cm.k_cq, cm.f_cq);
    const R srcw = kval<R>(cm.k_srcw, cm.f_srcw);
    R a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] = omq * U[k];
    a[0] = a[0] + srcw * B0;
    a[1] = a[1] + srcw * B1;
    // e_x-flux (X) and e_y-flux (Y) terms, sign included: omega/(2c) Phi
    const R X[6] = {-(cq * P[0]), -(cq * P[2]), -(cq * U[0]), R(0), -(cq * U[1]), R(0)};
    const R Y[6] = {-(cq * P[1]), -(cq * P[3]), R(0), -(cq * U[0]), R(0), -(cq * U[1])};
    constexpr bool hasX[6] = {true, true, true, false, true, false};
    constexpr bool hasY[6] = {true, true, false, true, false, true};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const R s0 = hasX[k] ? a[k] + X[k] : a[k];     // q0 = (1, 0)
        const R s2 = hasX[k] ? a[k] - X[k] : a[k];     // q2 = (-1, 0)
        const R s1 = hasY[k] ? a[k] + Y[k] : a[k];     // q1 = (0, 1)
        const R s3 = hasY[k] ? a[k] - Y[k] : a[k];     // q3 = (0, -1)
        out[0][k] = omc * g[0][k] + s0;
        out[1][k] = omc * g[1][k] + s1;
        out[2][k] = omc * g[2][k] + s2;
        out[3][k] = omc * g[3][k] + s3;
    }
}

// The state record of one node (lbm_record_bytes: v and F - I, 6 tiled planes).
template <typename R, bool SH>
__device__ __forceinline__ void write_record(void* record, int ntile, int x, int y, const R U[6]) {
    R* rec = (R*)record + tile_base(ntile, 6, x, y);
    rec[0] = U[0];
    rec[kTile] = U[1];
    rec[2 * kTile] = SH ? U[2] : U[2] - R(1);
    rec[3 * kTile] = U[3];
    rec[4 * kTile] = U[4];
    rec[5 * kTile] = SH ? U[5] : U[5] - R(1);
}

}  // namespace lbm
