// Forward kernels of the D2Q4 x 6 vectorial LBM on gfx950: the fused collide-stream step
// (Sec. 3.7), the traction-wall F^b solve (Sec. 3.6), the second-order initialisation
// (Sec. 3.4) and the recoveries from stored post-collision populations (Sec. 3.5).
//
// Layout: populations, u* and records in 64-node row tiles holding all their planes
// contiguously (tile_base in lbm_device.hpp).  One thread per node, one wavefront per
// tile, kTilesPerBlock tiles per workgroup; the tile order is remapped so that each of the
// eight XCDs sweeps a contiguous band of rows (its L2 then serves the one-element overlap
// of the x -/+ 1 pulls between adjacent tiles).  Each stored value is written once per
// pass, with non-temporal stores.
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"

namespace lbm {

// F^b of every link of the traction edges at step n -> n+1 (Sec. 3.6).  Reading of the
// extrapolation the paper leaves open: with X0 the wall node and X1 the first interior
// node, G = F_{.B} + (dt/2) d_B v (the kinematic identity moves F by half a step) and the
// tangential column is 3/2 G(X0) - 1/2 G(X1) (linear extrapolation to the half-way wall);
// the Newton guess for the normal column is 3/2 F_{.A}(X0) - 1/2 F_{.A}(X1).
//
// One launch covers every traction edge (each edge reads level n only and writes its own
// slice of the staging buffer), one wavefront per workgroup: the solve is latency-bound,
// so the links are spread over as many compute units as there are wavefronts.  Lane l of
// a wavefront recovers U at edge position s0 - 2 + l (wrapped on a periodic edge) on the
// wall row and the first interior row; lanes 2 .. 61 solve the links s0 .. s0 + 59 and
// take the velocities of their tangential stencil (central, or one-sided at the ends of
// an open edge: never more than two positions away) from the neighbouring lanes.  Each
// node is thus read once per wavefront instead of once per stencil use: on the edges
// normal to x every lane reads its own tile row, 24 separate cache lines per node.
// The edge's normal axis AX is a template parameter (fixed per edge, so per wavefront):
// with the axis known, F, the tangent and the per-node vectors index with constants and
// stay in registers.
template <int ST, int LAW, bool FIELDS, bool LINES, int AX>
__device__ __forceinline__ void traction_solve(const TractionArgs& a, int e) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const EdgeGeom G = edge_geom(e);
    const int L = (AX == 0) ? cm.ny : cm.nx;
    const bool per_t = (AX == 0) ? cm.periodic_y : cm.periodic_x;
    constexpr int Bx = 1 - AX;
    const int lane = int(threadIdx.x);
    const int s = (int(blockIdx.x) - a.eblk[e]) * kTracOut - 2 + lane;   // this lane's position
    const T* pop = (const T*)a.pop;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    const R hdt = R(0.5 * cm.dt);
    const R inv2h = R(1.0 / (2.0 * cm.dx));

    // U of level n at this lane's window position, wall row (r = 0) and first interior row
    int pw = s;
    bool have = true;
    if (per_t) pw = wrap_index(s, L);
    else have = s >= 0 && s < L;
    R Uw[2][6];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        if (have) {
            const XY nd = edge_node(G, cm.nx, cm.ny, r, pw);
            double b0, b1;
            body_at<FIELDS>(cm, nd.y * cm.nx + nd.x, n, a.r_n, b0, b1);
            if constexpr (LINES) {
                // level n+1 of the two-level step, from the wall lines of the staging buffer
                const T* lv = (const T*)wall_lines(a.aux, cm.nx, cm.ny).lines + line_slot(cm.nx, cm.ny, e, r, pw) * 24;
                recover_vals<T, R>(lv, 1, hdt * R(b0), hdt * R(b1), Uw[r]);
            } else {
                recover_node<T, R>(pop, cm.ntile, nd.x, nd.y, hdt * R(b0), hdt * R(b1), Uw[r]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) Uw[r][k] = R(0);
        }
    }

    // the stencil of the link at s, as lane offsets (a wrapped position is also held by the
    // lane at its unwrapped offset, so an offset beyond +-2 is taken modulo L)
    const bool solve = lane >= 2 && lane < kTracWin - 2 && s < L;
    Stencil sten = tangential_stencil(solve ? s : 0, L, per_t);
    int dl[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        int d = sten.p[j] - (solve ? s : 0);
        if (d > 2) d -= L;
        if (d < -2) d += L;
        dl[j] = solve ? d : 0;
    }
    R Vs[2][3][2];                     // velocity of row r at stencil entry j
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 2; ++k) Vs[r][j][k] = __shfl(Uw[r][k], lane + dl[j], kTracWin);
    if (!solve) return;

    R Ghat[2][2], Fa[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            R dv = R(0);
#pragma unroll
            for (int j = 0; j < 3; ++j) dv += R(sten.w[j]) * Vs[r][j][k];
            dv *= inv2h;
            Ghat[r][k] = Uw[r][2 + 2 * k + Bx] + hdt * dv;
            Fa[r][k] = Uw[r][2 + 2 * k + AX];
        }
    }
    R tang[2], acol[2], Tv[2];
    for (int k = 0; k < 2; ++k) {
        tang[k] = R(1.5) * Ghat[0][k] - R(0.5) * Ghat[1][k];
        acol[k] = R(1.5) * Fa[0][k] - R(0.5) * Fa[1][k];
        Tv[k] = edge_value<R>(a.ed, e, k, s, L);
    }
    const XY n0 = edge_node(G, cm.nx, cm.ny, 0, s);
    R mu, lam;
    params_at<FIELDS, R>(cm, n0.y * cm.nx + n0.x, mu, lam);
    const bool ok = newton_column<R, LAW, SH, AX>(R(G.NA), tang, Tv, mu, lam, law_consts<R>(cm), acol,
                                                 cm.newton_max_iter, R(cm.newton_tol));
    if (!ok) atomicOr(cm.fault, (uint32_t)LBM_FAULT_NEWTON);
    int off[4], len[4];
    edge_offsets(cm.nx, cm.ny, off, len);
    R* aux = (R*)a.aux + 4 * (int64_t)(off[e] + s);
    for (int k = 0; k < 2; ++k) {
        aux[2 * k + AX] = acol[k];
        aux[2 * k + Bx] = tang[k];
    }
}

template <int ST, int LAW, bool FIELDS, bool LINES>
__global__ void __launch_bounds__(kTracWin) traction_kernel(TractionArgs a) {
    int e = 0;
    while (e < 3 && int(blockIdx.x) >= a.eblk[e + 1]) ++e;
    if (e == LBM_XMIN || e == LBM_XMAX) traction_solve<ST, LAW, FIELDS, LINES, 0>(a, e);
    else traction_solve<ST, LAW, FIELDS, LINES, 1>(a, e);
}

// ---------------------------------------------------------------- the fused step

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

template <int ST, int LAW, bool WALLS, bool FIELDS>
__global__ void __launch_bounds__(kBlock) step_kernel(StepArgs a) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny, ntile = cm.ntile;
    int x, y;
    if (!tile_thread(nx, ny, ntile, x, y)) return;
    const int64_t n = int64_t(nx) * ny;
    const T* __restrict__ src = (const T*)a.src;
    T* __restrict__ dst = (T*)a.dst;
    const int idx = y * nx + x;
    const int64_t own = tile_base(ntile, 24, x, y);

    // pull sources: q0 (1,0) from (x-1, y), q1 (0,1) from (x, y-1), q2 (-1,0) from (x+1, y),
    // q3 (0,-1) from (x, y+1) (eq:streaming); a source beyond a wall is a missing link.
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    bool miss0 = false, miss1 = false, miss2 = false, miss3 = false;
    if (xm < 0) { if (WALLS && !cm.periodic_x) { miss0 = true; xm = x; } else xm = nx - 1; }
    if (xp >= nx) { if (WALLS && !cm.periodic_x) { miss2 = true; xp = x; } else xp = 0; }
    if (ym < 0) { if (WALLS && !cm.periodic_y) { miss1 = true; ym = y; } else ym = ny - 1; }
    if (yp >= ny) { if (WALLS && !cm.periodic_y) { miss3 = true; yp = y; } else yp = 0; }
    const int64_t sb[4] = {tile_base(ntile, 24, xm, y), tile_base(ntile, 24, x, ym),
                           tile_base(ntile, 24, xp, y), tile_base(ntile, 24, x, yp)};

    // x-neighbour pulls come from the own tile (but for one lane), so issue them first
    R g[4][6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        g[0][k] = R(src[sb[0] + k * kTile]);
        g[2][k] = R(src[sb[2] + (12 + k) * kTile]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        g[1][k] = R(src[sb[1] + (6 + k) * kTile]);
        g[3][k] = R(src[sb[3] + (18 + k) * kTile]);
    }

    if constexpr (WALLS) {
        if (miss0) wall_link<T, R>(cm, a.ed, a.aux, LBM_XMIN, y, src + own, kTile, g[0]);
        if (miss2) wall_link<T, R>(cm, a.ed, a.aux, LBM_XMAX, y, src + own, kTile, g[2]);
        if (miss1) wall_link<T, R>(cm, a.ed, a.aux, LBM_YMIN, x, src + own, kTile, g[1]);
        if (miss3) wall_link<T, R>(cm, a.ed, a.aux, LBM_YMAX, x, src + own, kTile, g[3]);
    }

    double bd0, bd1;
    body_at<FIELDS>(cm, idx, n, a.r_np1, bd0, bd1);
    R mu, lam;
    params_at<FIELDS, R>(cm, idx, mu, lam);
    const R dt = kval<R>(cm.dt, cm.f_dt);
    R out[4][6], U[6], J;
    collide_node<R, LAW, SH>(cm, g, R(bd0), R(bd1), mu, lam, out, U, J);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) store_stream(dst + own + (6 * q + k) * kTile, to_storage<T>(out[q][k]));

    // displacement quadrature u*^{n+2} = u*^{n+1} + dt v^{n+1} (eq:trapezoid-u)
    if (!a.ustar) {
        // replay for the adjoint: the accumulator is not needed
    } else if constexpr (ST == LBM_F64_PLAIN) {
        double* us = (double*)a.ustar + tile_base(ntile, 2, x, y);
        store_stream(us, us[0] + dt * U[0]);
        store_stream(us + kTile, us[kTile] + dt * U[1]);
    } else {
        // u* = U + S: S += dt v; at a block boundary S moves into U (ustar_refs)
        const UstarRefs r = ustar_refs(a.ustar, ntile, ny, x, y);
#pragma unroll
        for (int cpt = 0; cpt < 2; ++cpt) {
            const float sn = r.S[cpt * kTile] + float(dt * U[cpt]);
            if (a.fold) {
                store_stream(r.U + cpt * kTile, r.U[cpt * kTile] + double(sn));
                store_stream(r.S + cpt * kTile, 0.0f);
            } else {
                store_stream(r.S + cpt * kTile, sn);
            }
        }
    }

    if (a.record) write_record<R, SH>(a.record, ntile, x, y, U);

    bool nonfinite = false;
#pragma unroll
    for (int k = 0; k < 6; ++k) nonfinite |= !finite_r(U[k]);
    const bool jbad = J <= R(0);
    if (nonfinite || jbad)
        atomicOr(cm.fault, (jbad ? (uint32_t)LBM_FAULT_J : 0u) | (nonfinite ? (uint32_t)LBM_FAULT_NONFINITE : 0u));
}

// ---------------------------------------------------------------- two fused steps

// Pulled populations of node (x, y) from a stored level (eq:streaming, periodic wrap).
template <typename T, typename R>
__device__ __forceinline__ void pull_node(const T* __restrict__ src, int ntile, int nx, int ny, int x, int y,
                                          R g[4][6]) {
    const int xm = wrap_dec(x, nx), xp = wrap_inc(x, nx);
    const int ym = wrap_dec(y, ny), yp = wrap_inc(y, ny);
    const int64_t b0 = tile_base(ntile, 24, xm, y), b1 = tile_base(ntile, 24, x, ym);
    const int64_t b2 = tile_base(ntile, 24, xp, y), b3 = tile_base(ntile, 24, x, yp);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        g[0][k] = R(src[b0 + k * kTile]);
        g[1][k] = R(src[b1 + (6 + k) * kTile]);
        g[2][k] = R(src[b2 + (12 + k) * kTile]);
        g[3][k] = R(src[b3 + (18 + k) * kTile]);
    }
}

// The per-node tail of a two-level update at output node (x, y): the displacement
// quadrature over both levels (eq:trapezoid-u) with the accumulator updates and folds of two
// single steps, and the records of both levels.  spre: the node's block sums S, loaded
// earlier by the caller (shifted storages), or NULL to load them here.
template <int ST, bool REC>
__device__ __forceinline__ void pair_tail(const Step2Args& a, int x, int y, const typename Storage<ST>::real U1[6],
                                          const typename Storage<ST>::real U2[6], const float* spre) {
    using R = typename Storage<ST>::real;
    constexpr bool SH = Storage<ST>::shifted;
    const Common& cm = a.cm;
    const int ntile = cm.ntile;
    const R dt = kval<R>(cm.dt, cm.f_dt);
    if (!a.ustar) {
    } else if constexpr (ST == LBM_F64_PLAIN) {
        double* us = (double*)a.ustar + tile_base(ntile, 2, x, y);
        const double s0 = us[0] + dt * U1[0], s1 = us[kTile] + dt * U1[1];
        store_stream(us, s0 + dt * U2[0]);
        store_stream(us + kTile, s1 + dt * U2[1]);
    } else {
        const UstarRefs rf = ustar_refs(a.ustar, ntile, cm.ny, x, y);
#pragma unroll
        for (int cpt = 0; cpt < 2; ++cpt) {
            float sn = (spre ? spre[cpt] : rf.S[cpt * kTile]) + float(dt * U1[cpt]);
            bool moved = false;
            double u = 0.0;
            if (a.fold1) {
                u = rf.U[cpt * kTile] + double(sn);
                sn = 0.0f;
                moved = true;
            }
            sn = sn + float(dt * U2[cpt]);
            if (a.fold2) {
                u = (moved ? u : rf.U[cpt * kTile]) + double(sn);
                sn = 0.0f;
                moved = true;
            }
            if (moved) store_stream(rf.U + cpt * kTile, u);
            store_stream(rf.S + cpt * kTile, sn);
        }
    }
    if constexpr (REC) {
        if (a.record1) write_record<R, SH>(a.record1, ntile, x, y, U1);
        if (a.record2) write_record<R, SH>(a.record2, ntile, x, y, U2);
    }
}

// Level n+1 of a node on a wall line or first interior line into the wall lines of the
// staging buffer (every such line through it), and U^{n+1} of a wall-line node.
template <typename T, typename R>
__device__ __forceinline__ void store_wall_lines(const Common& cm, void* aux, int xg, int xc, int r, int yr,
                                                 const R f1[4][6], const R U1[6]) {
    const int nx = cm.nx, ny = cm.ny;
    const WallLines wl = wall_lines(aux, nx, ny);
    int off[4], len[4];
    edge_offsets(nx, ny, off, len);
    int er[4] = {-1, -1, -1, -1}, es[4] = {0, 0, 0, 0};
    if (!cm.periodic_x) {
        if (xg <= 1) { er[LBM_XMIN] = xg; es[LBM_XMIN] = yr; }
        if (xg >= nx - 2) { er[LBM_XMAX] = nx - 1 - xg; es[LBM_XMAX] = yr; }
    }
    if (!cm.periodic_y) {
        if (r <= 1) { er[LBM_YMIN] = r; es[LBM_YMIN] = xc; }
        if (r >= ny - 2) { er[LBM_YMAX] = ny - 1 - r; es[LBM_YMAX] = xc; }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (er[e] < 0) continue;
        T* lv = (T*)wl.lines + line_slot(nx, ny, e, er[e], es[e]) * 24;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 6; ++k) lv[6 * q + k] = T(f1[q][k]);
        if (er[e] == 0) {
            R* u = (R*)wl.u1 + (int64_t(off[e]) + es[e]) * 6;
#pragma unroll
            for (int k = 0; k < 6; ++k) u[k] = U1[k];
        }
    }
}

// Temporal blocking of the step: one pass takes f*^n to f*^{n+2} without storing level
// n+1.  A workgroup owns a block of kPairRows rows of one 64-node tile column (a
// strip).  Wave w < kPairWaves takes row y0 - 1 + w of the strip through level n+1,
// pulling level n straight from HBM; one more wave takes the two columns beside the strip
// (x = c0 - 1 and c0 + 64) through level n+1 on the block's rows.  The level n+1 values
// that cross rows go through LDS, those that cross columns inside the strip through lane
// shuffles, and waves 1 .. kPairRows take their row on to level n+2.  Every level n+1
// value that an output pulls is so computed in the workgroup (the edge rows and columns
// are computed by the neighbouring workgroups as well), and loads and stores are whole
// aligned tiles.  Each node's arithmetic is collide_node, as in step_kernel, and level
// n+1 is rounded to the storage type, so the result is bit for bit that of two single
// steps.  WALLS: the level-n links of wall nodes are rebuilt in the first level as
// step_kernel rebuilds them, the wall nodes are left out of the second level, and level
// n+1 of the wall lines goes to the staging buffer for step2_wall_kernel.
// The LDS of one two-level workgroup: level n+1 of the q1 and q3 planes of every row wave
// (read by the rows above and below) and of the nodes beside the strip (q0 at c0 - 1, q2
// at c0 + 64).
template <typename R>
struct PairLds {
    R xq1[kPairWaves][6][kTile];
    R xq3[kPairWaves][6][kTile];
    R xh[2][6][kPairRows];
};

template <int ST, int LAW, bool FIELDS, bool REC, bool WALLS>
__device__ __forceinline__ void step2_body(const Step2Args& a, int strip, int blk,
                                           PairLds<typename Storage<ST>::real>& sh) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    auto& xq1 = sh.xq1;
    auto& xq3 = sh.xq3;
    auto& xh = sh.xh;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny, ntile = cm.ntile;
    const int64_t n = int64_t(nx) * ny;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & (kTile - 1);
    const int c0 = strip * kTile, y0 = blk * kPairRows;
    const int r = y0 - 1 + w;
    const int xg = c0 + lane;
    const int xc = wrap_near(xg, nx);
    const int yr = wrap_near(r, ny);
    const T* __restrict__ src = (const T*)a.src;
    T* __restrict__ dst = (T*)a.dst;
    const int idx1 = yr * nx + xc;
    // a node of the grid (a lane or row beyond a wall is not; along a periodic axis every
    // lane and row is the node it wraps to)
    const bool valid = !WALLS || ((cm.periodic_x || xg < nx) && (cm.periodic_y || (r >= 0 && r < ny)));

    R f1[4][6], U1[6], g[4][6], mu, lam;
    R B2[2];                                  // r_np2 b(X) of this wave's node (level n+2)
    bool nonfinite = false, jbad = false;
    // the displacement block sums S of an inner wave's output node, loaded with level n so
    // that the load is in flight across the barrier (shifted storages)
    float spre[2] = {0.0f, 0.0f};
    if constexpr (ST != LBM_F64_PLAIN) {
        if (a.ustar && w >= 1 && w <= kPairRows && r < ny) {
            const float* S = ustar_refs(a.ustar, ntile, ny, xg, r).S;
            spre[0] = S[0];
            spre[1] = S[kTile];
        }
    }
    if (w < kPairWaves) {
        // level n -> n+1 on row r: q0 from x-1 and q2 from x+1 of row r (own lanes shifted,
        // the two end lanes from the columns beside the strip), q1 from row r-1, q3 from r+1
        const int64_t bo = tile_base(ntile, 24, xc, yr);
        const int64_t bm = tile_base(ntile, 24, xc, wrap_near(r - 1, ny));
        const int64_t bp = tile_base(ntile, 24, xc, wrap_near(r + 1, ny));
        R own0[6], own2[6], h[6] = {};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            own0[k] = R(src[bo + k * kTile]);
            own2[k] = R(src[bo + (12 + k) * kTile]);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            g[1][k] = R(src[bm + (6 + k) * kTile]);
            g[3][k] = R(src[bp + (18 + k) * kTile]);
        }
        if (lane == 0 || lane == kTile - 1) {
            const int64_t bh = lane == 0 ? tile_base(ntile, 24, wrap_near(c0 - 1, nx), yr)
                                         : tile_base(ntile, 24, wrap_near(c0 + kTile, nx), yr) + 12 * kTile;
#pragma unroll
            for (int k = 0; k < 6; ++k) h[k] = R(src[bh + k * kTile]);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const R up = __shfl_up(own0[k], 1), dn = __shfl_down(own2[k], 1);
            g[0][k] = lane == 0 ? h[k] : up;
            g[2][k] = lane == kTile - 1 ? h[k] : dn;
        }
        if constexpr (WALLS) {
            // the missing links of level n at wall nodes (eq:boundary-general), as in
            // step_kernel; lanes and rows beyond a wall hold no node and feed only wall
            // nodes, whose level n+2 the wall kernel computes
            if (valid) {
                if (!cm.periodic_x && xg == 0) wall_link<T, R>(cm, a.ed, a.aux, LBM_XMIN, yr, src + bo, kTile, g[0]);
                if (!cm.periodic_x && xg == nx - 1) wall_link<T, R>(cm, a.ed, a.aux, LBM_XMAX, yr, src + bo, kTile, g[2]);
                if (!cm.periodic_y && r == 0) wall_link<T, R>(cm, a.ed, a.aux, LBM_YMIN, xc, src + bo, kTile, g[1]);
                if (!cm.periodic_y && r == ny - 1) wall_link<T, R>(cm, a.ed, a.aux, LBM_YMAX, xc, src + bo, kTile, g[3]);
            }
        }
        R B1[2];
        body_r<FIELDS, R>(cm, idx1, n, a.r_np1, a.fb1, B1[0], B1[1]);
        body_r<FIELDS, R>(cm, idx1, n, a.r_np2, a.fb2, B2[0], B2[1]);
        params_at<FIELDS, R>(cm, idx1, mu, lam);
        R J1;
        collide_node<R, LAW, SH>(cm, g, B1[0], B1[1], mu, lam, f1, U1, J1);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 6; ++k) f1[q][k] = R(to_storage<T>(f1[q][k]));   // the stored value of level n+1
        if (valid) {
#pragma unroll
            for (int k = 0; k < 6; ++k) nonfinite |= !finite_r(U1[k]);
            jbad = J1 <= R(0);
        }
        if constexpr (WALLS) {
            if (valid) store_wall_lines<T, R>(cm, a.aux, xg, xc, r, yr, f1, U1);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            xq1[w][k][lane] = f1[1][k];
            xq3[w][k][lane] = f1[3][k];
            g[0][k] = __shfl_up(f1[0][k], 1);
            g[2][k] = __shfl_down(f1[2][k], 1);
        }
    } else {
        // the nodes beside the strip: lane j < kPairRows at (c0 - 1, y0 + j), lane
        // kPairRows + j at (c0 + 64, y0 + j); the other lanes repeat the last node
        const int j = min(lane, 2 * kPairRows - 1);
        const int side = j / kPairRows, row = j - side * kPairRows;
        const int hx = wrap_near(side == 0 ? c0 - 1 : c0 + kTile, nx), hy = wrap_near(y0 + row, ny);
        R gh[4][6], fh[4][6], Uh[6], Jh, muh, lamh;
        pull_node<T, R>(src, ntile, nx, ny, hx, hy, gh);
        if constexpr (WALLS) {
            const int hxg = side == 0 ? c0 - 1 : c0 + kTile, hyg = y0 + row;
            if ((cm.periodic_x || (hxg >= 0 && hxg < nx)) && (cm.periodic_y || hyg < ny)) {
                const T* hown = src + tile_base(ntile, 24, hx, hy);
                if (!cm.periodic_x && hx == 0) wall_link<T, R>(cm, a.ed, a.aux, LBM_XMIN, hy, hown, kTile, gh[0]);
                if (!cm.periodic_x && hx == nx - 1) wall_link<T, R>(cm, a.ed, a.aux, LBM_XMAX, hy, hown, kTile, gh[2]);
                if (!cm.periodic_y && hy == 0) wall_link<T, R>(cm, a.ed, a.aux, LBM_YMIN, hx, hown, kTile, gh[1]);
                if (!cm.periodic_y && hy == ny - 1) wall_link<T, R>(cm, a.ed, a.aux, LBM_YMAX, hx, hown, kTile, gh[3]);
            }
        }
        const int hidx = hy * nx + hx;
        R Bh0, Bh1;
        body_r<FIELDS, R>(cm, hidx, n, a.r_np1, a.fb1, Bh0, Bh1);
        params_at<FIELDS, R>(cm, hidx, muh, lamh);
        collide_node<R, LAW, SH>(cm, gh, Bh0, Bh1, muh, lamh, fh, Uh, Jh);
        if (lane < 2 * kPairRows) {
#pragma unroll
            for (int k = 0; k < 6; ++k) xh[side][k][row] = R(to_storage<T>(side == 0 ? fh[0][k] : fh[2][k]));
        }
    }
    __syncthreads();

    // level n+1 -> n+2 on row r for the inner waves
    const int xo = c0 + lane;
    if (w >= 1 && w <= kPairRows) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            g[1][k] = xq1[w - 1][k][lane];
            g[3][k] = xq3[w + 1][k][lane];
            // both end values are read by every lane (one address per wave) and selected
            // by value: a store guarded by the lane would let the compiler merge the two
            // into one write at a lane-dependent index of g, a select over all 24 entries
            const R e0 = xh[0][k][w - 1], e2 = xh[1][k][w - 1];
            g[0][k] = lane == 0 ? e0 : g[0][k];
            g[2][k] = lane == kTile - 1 ? e2 : g[2][k];
        }
        R f2[4][6], U2[6], J2;
        collide_node<R, LAW, SH>(cm, g, B2[0], B2[1], mu, lam, f2, U2, J2);
        const bool wall_node = WALLS && ((!cm.periodic_x && (xo == 0 || xo == nx - 1)) ||
                                         (!cm.periodic_y && (r == 0 || r == ny - 1)));
        if (r < ny && xo < nx && !wall_node) {
            const int64_t ob = tile_base(ntile, 24, xo, r);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < 6; ++k) store_stream(dst + ob + (6 * q + k) * kTile, to_storage<T>(f2[q][k]));
            pair_tail<ST, REC>(a, xo, r, U1, U2, ST != LBM_F64_PLAIN && a.ustar ? spre : nullptr);
#pragma unroll
            for (int k = 0; k < 6; ++k) nonfinite |= !finite_r(U2[k]);
            jbad |= J2 <= R(0);
        }
    }
    if (nonfinite || jbad)
        atomicOr(cm.fault, (jbad ? (uint32_t)LBM_FAULT_J : 0u) | (nonfinite ? (uint32_t)LBM_FAULT_NONFINITE : 0u));
}

template <int ST, int LAW, bool FIELDS, bool REC, bool WALLS>
__global__ void __launch_bounds__((kPairWaves + 1) * kTile) step2_kernel(Step2Args a) {
    __shared__ PairLds<typename Storage<ST>::real> sh;
    int strip, blk;
    pair_block(a.map, remap_tile(blockIdx.x, gridDim.x), strip, blk);
    step2_body<ST, LAW, FIELDS, REC, WALLS>(a, strip, blk, sh);
}

// The interior blocks (the periodic code) and the blocks along the walls (the wall code)
// of a walled grid in one launch, so that the few rim blocks fill the tail of the bulk
// instead of running as a launch of their own.  Every rim_period-th block of the order is
// a rim block while they last: each XCD's contiguous share of the order (remap_tile) then
// holds its share of them.  Each block computes what it computes in its own launch.
template <int ST, int LAW, bool FIELDS, bool REC>
__global__ void __launch_bounds__((kPairWaves + 1) * kTile) step2_split_kernel(Step2Args a) {
    __shared__ PairLds<typename Storage<ST>::real> sh;
    const int b = remap_tile(blockIdx.x, gridDim.x);
    const int p = a.rim_period;
    bool rim = false;
    int i = b;
    if (b < a.n_rim * p) {
        const int g = fdiv(b, a.d_rim_period), pos = b - g * p;
        rim = pos == p - 1;
        i = rim ? g : g * (p - 1) + pos;
    } else {
        i = a.n_rim * (p - 1) + (b - a.n_rim * p);
    }
    int strip, blk;
    if (rim) {
        pair_block(a.map2, i, strip, blk);
        step2_body<ST, LAW, FIELDS, REC, true>(a, strip, blk, sh);
    } else {
        pair_block(a.map, i, strip, blk);
        step2_body<ST, LAW, FIELDS, REC, false>(a, strip, blk, sh);
    }
}

// Level n+1 -> n+2 at the wall nodes of a two-level step on a grid with walls: one thread
// per link slot of the staging buffer (a corner node is taken by the first of its edges).
// Level n+1 comes from the wall lines, F^b^{n+1} from the staging buffer (written by the
// traction kernel from the same lines), the wall data of t^{n+3/2} from ed2; the arithmetic
// is that of step_kernel at a wall node (collide_node, wall_link), the tail that of the
// two-level kernel (pair_tail).
template <int ST, int LAW, bool FIELDS, bool REC>
__global__ void __launch_bounds__(kTile) step2_wall_kernel(Step2Args a) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny;
    // the edge of this link slot (selected without arrays indexed by a lane-dependent edge,
    // which would go to scratch memory)
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * ny + 2 * nx) return;
    const int e = t < ny ? LBM_XMIN : t < 2 * ny ? LBM_XMAX : t < 2 * ny + nx ? LBM_YMIN : LBM_YMAX;
    const int bce = e == LBM_XMIN ? cm.bc[LBM_XMIN] : e == LBM_XMAX ? cm.bc[LBM_XMAX]
                  : e == LBM_YMIN ? cm.bc[LBM_YMIN] : cm.bc[LBM_YMAX];
    if (bce == LBM_PERIODIC) return;
    const int s = t - edge_off(nx, ny, e);
    const XY nd = edge_node(edge_geom(e), nx, ny, 0, s);
    const int x = nd.x, y = nd.y;
    const bool on[4] = {!cm.periodic_x && x == 0, !cm.periodic_x && x == nx - 1,
                        !cm.periodic_y && y == 0, !cm.periodic_y && y == ny - 1};
    // a corner taken by an earlier edge
    if ((e > LBM_XMIN && on[LBM_XMIN]) || (e > LBM_XMAX && on[LBM_XMAX]) || (e > LBM_YMIN && on[LBM_YMIN])) return;
    const WallLines wl = wall_lines(a.aux, nx, ny);
    const T* lines = (const T*)wl.lines;
    const T* ownp = lines + line_slot(nx, ny, e, 0, s) * 24;
    // pulls from the lines: q0 from (x-1, y), q1 from (x, y-1), q2 from (x+1, y), q3 from (x, y+1)
    R g[4][6];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool miss = on[q == 0 ? LBM_XMIN : q == 1 ? LBM_YMIN : q == 2 ? LBM_XMAX : LBM_YMAX];
        if (miss) continue;
        const int sx = wrap_index(x - dir_i(q), nx), sy = wrap_index(y - dir_j(q), ny);
        int le = 0, lr = 0, ls = 0;
        find_line(cm, sx, sy, le, lr, ls);
        const T* sp = lines + line_slot(nx, ny, le, lr, ls) * 24;
#pragma unroll
        for (int k = 0; k < 6; ++k) g[q][k] = R(sp[6 * q + k]);
    }
    if (on[LBM_XMIN]) wall_link<T, R>(cm, a.ed2, a.aux, LBM_XMIN, y, ownp, 1, g[0]);
    if (on[LBM_XMAX]) wall_link<T, R>(cm, a.ed2, a.aux, LBM_XMAX, y, ownp, 1, g[2]);
    if (on[LBM_YMIN]) wall_link<T, R>(cm, a.ed2, a.aux, LBM_YMIN, x, ownp, 1, g[1]);
    if (on[LBM_YMAX]) wall_link<T, R>(cm, a.ed2, a.aux, LBM_YMAX, x, ownp, 1, g[3]);
    const int64_t n = int64_t(nx) * ny;
    const int idx = y * nx + x;
    double bd0, bd1;
    body_at<FIELDS>(cm, idx, n, a.r_np2, bd0, bd1);
    R mu, lam;
    params_at<FIELDS, R>(cm, idx, mu, lam);
    R f2[4][6], U2[6], J2;
    collide_node<R, LAW, SH>(cm, g, R(bd0), R(bd1), mu, lam, f2, U2, J2);
    T* dst = (T*)a.dst + tile_base(cm.ntile, 24, x, y);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) store_stream(dst + (6 * q + k) * kTile, to_storage<T>(f2[q][k]));
    R U1[6];
    const R* u1 = (const R*)wl.u1 + (int64_t(edge_off(nx, ny, e)) + s) * 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) U1[k] = u1[k];
    pair_tail<ST, REC>(a, x, y, U1, U2, nullptr);
    bool nonfinite = false;
#pragma unroll
    for (int k = 0; k < 6; ++k) nonfinite |= !finite_r(U2[k]);
    const bool jbad = J2 <= R(0);
    if (nonfinite || jbad)
        atomicOr(cm.fault, (jbad ? (uint32_t)LBM_FAULT_J : 0u) | (nonfinite ? (uint32_t)LBM_FAULT_NONFINITE : 0u));
}

// ---------------------------------------------------------------- recoveries

template <int ST, bool FIELDS, int MODE>   // MODE 0 moments (double), 1 record (R), 2 displacement
__global__ void __launch_bounds__(kBlock) recover_kernel(RecoverArgs a) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = int(idx / cm.nx), x = int(idx - int64_t(y) * cm.nx);
    double b0, b1;
    body_at<FIELDS>(cm, (int)idx, n, a.r_n, b0, b1);
    const double hdt = 0.5 * cm.dt;
    R U[6];
    recover_node<T, R>((const T*)a.pop, cm.ntile, x, y, R(hdt * b0), R(hdt * b1), U);
    if constexpr (MODE == 0) {
        double* out = (double*)a.out;
        for (int k = 0; k < 6; ++k) {
            double v = double(U[k]);
            if (!SH && (k == 2 || k == 5)) v -= 1.0;
            out[k * n + idx] = v;
        }
    } else if constexpr (MODE == 1) {
        R* out = (R*)a.out + tile_base(cm.ntile, 6, x, y);
        for (int k = 0; k < 6; ++k) {
            R v = U[k];
            if (!SH && (k == 2 || k == 5)) v -= R(1);
            out[k * kTile] = v;
        }
    } else {
        double* out = (double*)a.out;
        for (int cpt = 0; cpt < 2; ++cpt) {
            double ustar;
            if constexpr (ST == LBM_F64_PLAIN) {
                ustar = ((const double*)a.ustar)[tile_base(cm.ntile, 2, x, y) + cpt * kTile];
            } else {
                const UstarRefs r = ustar_refs(const_cast<void*>(a.ustar), cm.ntile, cm.ny, x, y);
                ustar = r.U[cpt * kTile] + double(r.S[cpt * kTile]);
            }
            out[cpt * n + idx] = ustar - hdt * double(U[cpt]);
        }
    }
}

// ---------------------------------------------------------------- stresses

// P(F) and sigma = J^{-1} P F^T (Sec. 3.5) of the recovered state, in FP64 from the
// stored populations (shifted evaluation for every storage: F - I is formed first).
template <int ST, int LAW, bool FIELDS>
__global__ void __launch_bounds__(kBlock) stress_kernel(RecoverArgs a) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = int(idx / cm.nx), x = int(idx - int64_t(y) * cm.nx);
    double b0, b1;
    body_at<FIELDS>(cm, (int)idx, n, a.r_n, b0, b1);
    const double hdt = 0.5 * cm.dt;
    R U[6];
    recover_node<T, R>((const T*)a.pop, cm.ntile, x, y, R(hdt * b0), R(hdt * b1), U);
    double ft[4] = {double(U[2]), double(U[3]), double(U[4]), double(U[5])};
    if (!SH) { ft[0] -= 1.0; ft[3] -= 1.0; }
    double mu, lam;
    params_at<FIELDS, double>(cm, (int)idx, mu, lam);
    double P[4], J;
    piola<double, LAW, true>(ft, mu, lam, law_consts<double>(cm), P, J);
    double* Po = (double*)a.out;
    for (int k = 0; k < 4; ++k) Po[k * n + idx] = P[k];
    if (a.out2) {
        const double F[4] = {1.0 + ft[0], ft[1], ft[2], 1.0 + ft[3]};
        const double iJ = 1.0 / J;
        double* So = (double*)a.out2;
        So[idx] = iJ * (P[0] * F[0] + P[1] * F[1]);
        So[n + idx] = iJ * (P[0] * F[2] + P[1] * F[3]);
        So[2 * n + idx] = iJ * (P[2] * F[2] + P[3] * F[3]);
    }
}

// ---------------------------------------------------------------- diagnostics

template <int ST, int LAW, bool FIELDS>
__global__ void __launch_bounds__(kBlock) diag_kernel(RecoverArgs a) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    double acc[LBM_DIAG_COUNT];
    for (int k = 0; k < LBM_DIAG_COUNT; ++k) acc[k] = 0.0;
    acc[7] = 1e300;
    acc[8] = 0.0;
    acc[9] = 0.0;
    const double hdt = 0.5 * cm.dt;
    // 1-degree rotation for the direction scan of the acoustic tensor
    const R cd = R(0.99984769515639123916), sd = R(0.017452406437283512820);
    for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < n;
         idx += int64_t(gridDim.x) * blockDim.x) {
        const int y = int(idx / cm.nx), x = int(idx - int64_t(y) * cm.nx);
        double b0, b1;
        body_at<FIELDS>(cm, (int)idx, n, a.r_n, b0, b1);
        R U[6];
        recover_node<T, R>((const T*)a.pop, cm.ntile, x, y, R(hdt * b0), R(hdt * b1), U);
        R mu, lam;
        params_at<FIELDS, R>(cm, (int)idx, mu, lam);
        R ft[4] = {U[2], U[3], U[4], U[5]};
        if (!SH) { ft[0] -= R(1); ft[3] -= R(1); }
        acc[0] += double(U[0]);
        acc[1] += double(U[1]);
        for (int k = 0; k < 4; ++k) acc[2 + k] += double(ft[k]);
        const R W = energy<R, LAW, true>(ft, mu, lam, law_consts<R>(cm));
        acc[6] += double(R(0.5) * (U[0] * U[0] + U[1] * U[1]) + W);
        const R J = R(1) + ft[0] + ft[3] + (ft[0] * ft[3] - ft[1] * ft[2]);
        acc[7] = fmin(acc[7], double(J));
        acc[8] = fmax(acc[8], double(sqrt_r(ft[0] * ft[0] + ft[1] * ft[1] + ft[2] * ft[2] + ft[3] * ft[3])));
        R C[16];
        tangent<R, LAW, true>(ft, mu, lam, law_consts<R>(cm), C);
        R cs = R(1), sn = R(0), best = R(0);
        for (int t = 0; t < 180; ++t) {
            const R nn[2] = {cs, sn};
            R Q[4];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 2; ++k) {
                    R v = R(0);
                    for (int A = 0; A < 2; ++A)
                        for (int B = 0; B < 2; ++B) v += nn[A] * C[8 * i + 4 * A + 2 * k + B] * nn[B];
                    Q[2 * i + k] = v;
                }
            const R tr = R(0.5) * (Q[0] + Q[3]);
            const R dd = R(0.5) * (Q[0] - Q[3]);
            const R off = R(0.5) * (Q[1] + Q[2]);
            const R lmax = tr + sqrt_r(dd * dd + off * off);
            best = best > lmax ? best : lmax;
            const R c2 = cs * cd - sn * sd;
            sn = sn * cd + cs * sd;
            cs = c2;
        }
        acc[9] = fmax(acc[9], double(sqrt_r(best)) / cm.c);
    }
    acc[6] *= cm.dx * cm.dx;
    // block reduction in FP64
    __shared__ double red[kBlock];
    double* part = (double*)a.scratch + int64_t(blockIdx.x) * LBM_DIAG_COUNT;
    for (int k = 0; k < LBM_DIAG_COUNT; ++k) {
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                const double o = red[threadIdx.x + w];
                double& m = red[threadIdx.x];
                m = (k == 7) ? fmin(m, o) : (k >= 8 ? fmax(m, o) : m + o);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) part[k] = red[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) diag_final_kernel(const double* part, int nblocks, double* out) {
    __shared__ double red[kBlock];
    for (int k = 0; k < LBM_DIAG_COUNT; ++k) {
        double m = (k == 7) ? 1e300 : 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
            const double o = part[b * LBM_DIAG_COUNT + k];
            m = (k == 7) ? fmin(m, o) : (k >= 8 ? fmax(m, o) : m + o);
        }
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                const double o = red[threadIdx.x + w];
                double& r = red[threadIdx.x];
                r = (k == 7) ? fmin(r, o) : (k >= 8 ? fmax(r, o) : r + o);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- initialisation

// U0 = (v0, F - I) as 6 double planes, F - I = (Fbar - I) + grad u0 by second-order
// differences.
__global__ void __launch_bounds__(kBlock) init_state_kernel(InitArgs a) {
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny;
    const int64_t n = int64_t(nx) * ny;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = int(idx / nx), x = int(idx - int64_t(y) * nx);
    double* U0 = (double*)a.scratch;
    U0[idx] = a.v0[idx];
    U0[n + idx] = a.v0[n + idx];
    const double inv2h = 1.0 / (2.0 * cm.dx);
    for (int cpt = 0; cpt < 2; ++cpt) {
        double gx = 0.0, gy = 0.0;
        if (a.u0) {
            const double* u = a.u0 + cpt * n;
            gx = fd_along<double>([&](int s) { return u[int64_t(y) * nx + s]; }, x, nx, cm.periodic_x, inv2h);
            gy = fd_along<double>([&](int s) { return u[int64_t(s) * nx + x]; }, y, ny, cm.periodic_y, inv2h);
        }
        U0[(2 + 2 * cpt) * n + idx] = (a.Fbar[2 * cpt] - (cpt == 0 ? 1.0 : 0.0)) + gx;
        U0[(3 + 2 * cpt) * n + idx] = (a.Fbar[2 * cpt + 1] - (cpt == 1 ? 1.0 : 0.0)) + gy;
    }
}

// Second-order populations (eq:init-compact with eq:init-Zq-components, eq:init-deltaPq,
// eq:init-expanded) in FP64 shifted form, then the first collision (level 0) and u*^1.
template <int ST, int LAW, bool FIELDS>
__global__ void __launch_bounds__(kBlock) init_pop_kernel(InitArgs a) {
    using Tr = Storage<ST>;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny;
    const int64_t n = int64_t(nx) * ny;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = int(idx / nx), x = int(idx - int64_t(y) * nx);
    const double* U0p = (const double*)a.scratch;
    const double c = cm.c, dt = cm.dt, hdt = 0.5 * cm.dt;
    const double inv2h = 1.0 / (2.0 * cm.dx);
    double U0[6], dX[6], dY[6];
    for (int k = 0; k < 6; ++k) {
        const double* pl = U0p + k * n;
        U0[k] = pl[idx];
        dX[k] = fd_along<double>([&](int s) { return pl[int64_t(y) * nx + s]; }, x, nx, cm.periodic_x, inv2h);
        dY[k] = fd_along<double>([&](int s) { return pl[int64_t(s) * nx + x]; }, y, ny, cm.periodic_y, inv2h);
    }
    double mu, lam, b0, b1;
    params_at<FIELDS, double>(cm, (int)idx, mu, lam);
    body_at<FIELDS>(cm, (int)idx, n, a.r0, b0, b1);
    double C[16], P0[4], J;
    tangent<double, LAW, true>(&U0[2], mu, lam, law_consts<double>(cm), C);
    piola<double, LAW, true>(&U0[2], mu, lam, law_consts<double>(cm), P0, J);
    // d_alpha P = C : d_alpha F
    double dPX[4], dPY[4];
    for (int iA = 0; iA < 4; ++iA) {
        double sx = 0.0, sy = 0.0;
        for (int kB = 0; kB < 4; ++kB) {
            sx += C[4 * iA + kB] * dX[2 + kB];
            sy += C[4 * iA + kB] * dY[2 + kB];
        }
        dPX[iA] = sx;
        dPY[iA] = sy;
    }
    const double PhiX[6] = {-P0[0], -P0[2], -U0[0], 0.0, -U0[1], 0.0};
    const double PhiY[6] = {-P0[1], -P0[3], 0.0, -U0[0], 0.0, -U0[1]};
    double g0[4][6];
    for (int q = 0; q < 4; ++q) {
        const double i = dir_i(q), j = dir_j(q);
        double Z[6];
        Z[0] = b0 + dPX[0] + dPY[1] + c * (i * dX[0] + j * dY[0]);
        Z[1] = b1 + dPX[2] + dPY[3] + c * (i * dX[1] + j * dY[1]);
        Z[2] = dX[0] + c * (i * dX[2] + j * dY[2]);
        Z[3] = dY[0] + c * (i * dX[3] + j * dY[3]);
        Z[4] = dX[1] + c * (i * dX[4] + j * dY[4]);
        Z[5] = dY[1] + c * (i * dX[5] + j * dY[5]);
        double dP[4];
        for (int iA = 0; iA < 4; ++iA) {
            double sacc = 0.0;
            for (int kB = 0; kB < 4; ++kB) sacc += C[4 * iA + kB] * Z[2 + kB];
            dP[iA] = sacc;
        }
        const double D[6] = {
            0.25 * (Z[0] - (2.0 / c) * (i * dP[0] + j * dP[1])),
            0.25 * (Z[1] - (2.0 / c) * (i * dP[2] + j * dP[3])),
            0.25 * (Z[2] - (2.0 * i / c) * Z[0]),
            0.25 * (Z[3] - (2.0 * j / c) * Z[0]),
            0.25 * (Z[4] - (2.0 * i / c) * Z[1]),
            0.25 * (Z[5] - (2.0 * j / c) * Z[1]),
        };
        for (int k = 0; k < 6; ++k) {
            const double feq = 0.25 * (U0[k] + (2.0 / c) * (i * PhiX[k] + j * PhiY[k]));
            g0[q][k] = feq - hdt * D[k];
        }
    }
    // first collision at level 0 (eq:moment-U, eq:collision)
    double U[6];
    for (int k = 0; k < 6; ++k) U[k] = g0[0][k] + g0[1][k] + g0[2][k] + g0[3][k];
    U[0] += hdt * b0;
    U[1] += hdt * b1;
    double P[4];
    piola<double, LAW, true>(&U[2], mu, lam, law_consts<double>(cm), P, J);
    const double QX[6] = {-P[0], -P[2], -U[0], 0.0, -U[1], 0.0};
    const double QY[6] = {-P[1], -P[3], 0.0, -U[0], 0.0, -U[1]};
    const double srcw = dt * (2.0 - cm.omega) * 0.125;
    T* dst = (T*)a.dst + tile_base(cm.ntile, 24, x, y);
    for (int q = 0; q < 4; ++q) {
        const double i = dir_i(q), j = dir_j(q);
        for (int k = 0; k < 6; ++k) {
            const double feq = 0.25 * (U[k] + (2.0 / c) * (i * QX[k] + j * QY[k]));
            double v = g0[q][k] + cm.omega * (feq - g0[q][k]);
            if (k == 0) v += srcw * b0;
            if (k == 1) v += srcw * b1;
            if (!SH && (k == 2 || k == 5)) v += 0.25;
            dst[(6 * q + k) * kTile] = T(v);
        }
    }
    // u*^1 = u0 - (dt/2) v0 + dt v^0 (eq:trapezoid-u)
    for (int cpt = 0; cpt < 2; ++cpt) {
        const double u0 = a.u0 ? a.u0[cpt * n + idx] : 0.0;
        const double us1 = u0 - hdt * a.v0[cpt * n + idx] + dt * U[cpt];
        if constexpr (ST == LBM_F64_PLAIN) {
            ((double*)a.ustar)[tile_base(cm.ntile, 2, x, y) + cpt * kTile] = us1;
        } else {
            const UstarRefs r = ustar_refs(a.ustar, cm.ntile, cm.ny, x, y);
            r.U[cpt * kTile] = us1;
            r.S[cpt * kTile] = 0.0f;
        }
    }
    bool bad = !(J > 0.0);
    if (bad) atomicOr(cm.fault, (uint32_t)LBM_FAULT_J);
}

// ---------------------------------------------------------------- dispatch

static inline unsigned nblocks(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

template <int ST, int LAW>
static hipError_t step_st_law(const StepArgs& a, hipStream_t s) {
    const bool walls = !(a.cm.periodic_x && a.cm.periodic_y);
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    const dim3 grid(unsigned((int64_t(a.cm.ntile) * a.cm.ny + kTilesPerBlock - 1) / kTilesPerBlock));
    const dim3 block(kTile * kTilesPerBlock);
    if (walls) {
        if (fields) hipLaunchKernelGGL((step_kernel<ST, LAW, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<ST, LAW, true, false>), grid, block, 0, s, a);
    } else {
        if (fields) hipLaunchKernelGGL((step_kernel<ST, LAW, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<ST, LAW, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int ST>
static hipError_t step_st(const StepArgs& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: return step_st_law<ST, LBM_LOGNH>(a, s);
        case LBM_NH: return step_st_law<ST, LBM_NH>(a, s);
        case LBM_MR: return step_st_law<ST, LBM_MR>(a, s);
        case LBM_YEOH: return step_st_law<ST, LBM_YEOH>(a, s);
        case LBM_GENT: return step_st_law<ST, LBM_GENT>(a, s);
        default: return step_st_law<ST, LBM_SVK>(a, s);
    }
}

// The two-level bulk launch.  On a grid with walls, the blocks whose level-(n+1) region
// keeps two nodes away from every wall line run the periodic instantiation (no wall code:
// compiled in, the wall branches cost every node about a sixth of its speed), and only the
// blocks along the walls run the wall instantiation.
template <int ST, int LAW, bool FIELDS, bool REC>
static void step2_launch(const Step2Args& a0, hipStream_t s, bool walls) {
    const dim3 block((kPairWaves + 1) * kTile);
    const int nstrip = a0.nstrip, nblk = (a0.cm.ny + kPairRows - 1) / kPairRows;
    auto go = [&](const PairMap& m, bool w) {
        const int64_t nb = pair_map_blocks(m);
        if (nb <= 0) return;
        Step2Args a = a0;
        a.map = m;
        if (w) hipLaunchKernelGGL((step2_kernel<ST, LAW, FIELDS, REC, true>), dim3(unsigned(nb)), block, 0, s, a);
        else hipLaunchKernelGGL((step2_kernel<ST, LAW, FIELDS, REC, false>), dim3(unsigned(nb)), block, 0, s, a);
    };
    if (!walls) {
        go(pair_map(nstrip, nblk, 0, nstrip, 0, nblk), false);
        return;
    }
    // interior: columns c0 - 1 .. c0 + 64 within [2, nx - 3], rows y0 - 1 .. y0 + R within
    // [2, ny - 3] along each axis with walls
    int s_lo = 0, s_hi = nstrip, b_lo = 0, b_hi = nblk;
    if (!a0.cm.periodic_x) {
        s_lo = 1;
        s_hi = a0.cm.nx - 3 - kTile >= 0 ? (a0.cm.nx - 3 - kTile) / kTile + 1 : 0;
    }
    if (!a0.cm.periodic_y) {
        b_lo = (3 + kPairRows - 1) / kPairRows;
        b_hi = a0.cm.ny - 3 - kPairRows >= 0 ? (a0.cm.ny - 3 - kPairRows) / kPairRows + 1 : 0;
    }
    if (s_hi <= s_lo || b_hi <= b_lo) {
        go(pair_map(nstrip, nblk, 0, nstrip, 0, nblk), true);
        return;
    }
    const PairMap inner = pair_map(nstrip, nblk, s_lo, s_hi, b_lo, b_hi);
    PairMap rim = inner;
    rim.mode = 1;
    const int64_t n_in = pair_map_blocks(inner), n_rim = pair_map_blocks(rim);
    // FP64 keeps two launches: holding both codes costs its kernel an occupancy step
    if (ST == LBM_F64_PLAIN || n_rim <= 0) {
        go(inner, false);
        go(rim, true);
        return;
    }
    Step2Args a = a0;
    a.map = inner;
    a.map2 = rim;
    a.n_rim = int(n_rim);
    a.rim_period = int((n_in + n_rim) / n_rim);
    a.d_rim_period = fast_div(a.rim_period);
    if constexpr (ST != LBM_F64_PLAIN)
        hipLaunchKernelGGL((step2_split_kernel<ST, LAW, FIELDS, REC>), dim3(unsigned(n_in + n_rim)), block, 0, s, a);
}

template <int ST, int LAW>
static hipError_t step2_st_law(const Step2Args& a, hipStream_t s) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    const bool walls = !(a.cm.periodic_x && a.cm.periodic_y);
    // the record writes are compiled in only where asked for: their mere presence costs the
    // plain kernel about a tenth of its speed
    const bool rec = a.record1 || a.record2;
    if (a.wall_pass) {
        // one wavefront per workgroup: the pass is latency-bound, so its few thousand
        // links are spread over as many compute units as there are wavefronts
        const int links = 2 * a.cm.nx + 2 * a.cm.ny;
        const dim3 grid(unsigned((links + kTile - 1) / kTile)), block(kTile);
        if (fields) {
            if (rec) hipLaunchKernelGGL((step2_wall_kernel<ST, LAW, true, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((step2_wall_kernel<ST, LAW, true, false>), grid, block, 0, s, a);
        } else {
            if (rec) hipLaunchKernelGGL((step2_wall_kernel<ST, LAW, false, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((step2_wall_kernel<ST, LAW, false, false>), grid, block, 0, s, a);
        }
        return hipGetLastError();
    }
    if (fields) {
        if (rec) step2_launch<ST, LAW, true, true>(a, s, walls);
        else step2_launch<ST, LAW, true, false>(a, s, walls);
    } else {
        if (rec) step2_launch<ST, LAW, false, true>(a, s, walls);
        else step2_launch<ST, LAW, false, false>(a, s, walls);
    }
    return hipGetLastError();
}

template <int ST>
static hipError_t step2_st(const Step2Args& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: return step2_st_law<ST, LBM_LOGNH>(a, s);
        case LBM_NH: return step2_st_law<ST, LBM_NH>(a, s);
        case LBM_MR: return step2_st_law<ST, LBM_MR>(a, s);
        case LBM_YEOH: return step2_st_law<ST, LBM_YEOH>(a, s);
        case LBM_GENT: return step2_st_law<ST, LBM_GENT>(a, s);
        default: return step2_st_law<ST, LBM_SVK>(a, s);
    }
}

hipError_t launch_step2(const Step2Args& a, hipStream_t s) {
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: return step2_st<LBM_F32_SHIFTED>(a, s);
        case LBM_F16_SHIFTED: return step2_st<LBM_F16_SHIFTED>(a, s);
        default: return step2_st<LBM_F64_PLAIN>(a, s);
    }
}

hipError_t launch_step(const StepArgs& a, hipStream_t s) {
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: return step_st<LBM_F32_SHIFTED>(a, s);
        case LBM_F16_SHIFTED: return step_st<LBM_F16_SHIFTED>(a, s);
        default: return step_st<LBM_F64_PLAIN>(a, s);
    }
}

template <int ST, int LAW>
static hipError_t traction_st_law(const TractionArgs& a, hipStream_t s) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    const dim3 grid(unsigned(a.eblk[4])), block(kTracWin);
    if (a.lines) {
        if (fields) hipLaunchKernelGGL((traction_kernel<ST, LAW, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((traction_kernel<ST, LAW, false, true>), grid, block, 0, s, a);
    } else {
        if (fields) hipLaunchKernelGGL((traction_kernel<ST, LAW, true, false>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((traction_kernel<ST, LAW, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <int ST>
static hipError_t traction_st(const TractionArgs& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: return traction_st_law<ST, LBM_LOGNH>(a, s);
        case LBM_NH: return traction_st_law<ST, LBM_NH>(a, s);
        case LBM_MR: return traction_st_law<ST, LBM_MR>(a, s);
        case LBM_YEOH: return traction_st_law<ST, LBM_YEOH>(a, s);
        case LBM_GENT: return traction_st_law<ST, LBM_GENT>(a, s);
        default: return traction_st_law<ST, LBM_SVK>(a, s);
    }
}

hipError_t launch_traction(TractionArgs a, hipStream_t s) {
    // workgroup ranges of the traction edges; nothing to launch without one
    a.eblk[0] = 0;
    for (int e = 0; e < 4; ++e) {
        const int L = (e == LBM_XMIN || e == LBM_XMAX) ? a.cm.ny : a.cm.nx;
        a.eblk[e + 1] = a.eblk[e] + (a.cm.bc[e] == LBM_TRACTION ? (L + kTracOut - 1) / kTracOut : 0);
    }
    if (a.eblk[4] == 0) return hipSuccess;
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: return traction_st<LBM_F32_SHIFTED>(a, s);
        case LBM_F16_SHIFTED: return traction_st<LBM_F16_SHIFTED>(a, s);
        default: return traction_st<LBM_F64_PLAIN>(a, s);
    }
}

template <int MODE>
static hipError_t recover_dispatch(const RecoverArgs& a, hipStream_t s) {
    const bool fields = a.cm.body != nullptr;
    const dim3 grid(nblocks(int64_t(a.cm.nx) * a.cm.ny));
#define LBM_RECOVER(ST_)                                                                         \
    if (fields) hipLaunchKernelGGL((recover_kernel<ST_, true, MODE>), grid, dim3(kBlock), 0, s, a); \
    else hipLaunchKernelGGL((recover_kernel<ST_, false, MODE>), grid, dim3(kBlock), 0, s, a);
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: { LBM_RECOVER(LBM_F32_SHIFTED) break; }
        case LBM_F16_SHIFTED: { LBM_RECOVER(LBM_F16_SHIFTED) break; }
        default: { LBM_RECOVER(LBM_F64_PLAIN) break; }
    }
#undef LBM_RECOVER
    return hipGetLastError();
}

hipError_t launch_moments(const RecoverArgs& a, hipStream_t s) { return recover_dispatch<0>(a, s); }
hipError_t launch_record(const RecoverArgs& a, hipStream_t s) { return recover_dispatch<1>(a, s); }
hipError_t launch_displacement(const RecoverArgs& a, hipStream_t s) { return recover_dispatch<2>(a, s); }

template <int ST, int LAW>
static void stress_st_law(const RecoverArgs& a, hipStream_t s) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    const dim3 grid(nblocks(int64_t(a.cm.nx) * a.cm.ny));
    if (fields) hipLaunchKernelGGL((stress_kernel<ST, LAW, true>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((stress_kernel<ST, LAW, false>), grid, dim3(kBlock), 0, s, a);
}

template <int ST>
static void stress_st(const RecoverArgs& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: stress_st_law<ST, LBM_LOGNH>(a, s); break;
        case LBM_NH: stress_st_law<ST, LBM_NH>(a, s); break;
        case LBM_MR: stress_st_law<ST, LBM_MR>(a, s); break;
        case LBM_YEOH: stress_st_law<ST, LBM_YEOH>(a, s); break;
        case LBM_GENT: stress_st_law<ST, LBM_GENT>(a, s); break;
        default: stress_st_law<ST, LBM_SVK>(a, s); break;
    }
}

hipError_t launch_stress(const RecoverArgs& a, hipStream_t s) {
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: stress_st<LBM_F32_SHIFTED>(a, s); break;
        case LBM_F16_SHIFTED: stress_st<LBM_F16_SHIFTED>(a, s); break;
        default: stress_st<LBM_F64_PLAIN>(a, s); break;
    }
    return hipGetLastError();
}

template <int ST, int LAW>
static void diag_st_law(const RecoverArgs& a, hipStream_t s) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    const int64_t n = int64_t(a.cm.nx) * a.cm.ny;
    const unsigned nb = unsigned(std::min<int64_t>(kDiagBlocks, (n + kBlock - 1) / kBlock));
    if (fields) hipLaunchKernelGGL((diag_kernel<ST, LAW, true>), dim3(nb), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((diag_kernel<ST, LAW, false>), dim3(nb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kBlock), 0, s, (const double*)a.scratch, (int)nb,
                       (double*)a.out);
}

template <int ST>
static void diag_st(const RecoverArgs& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: diag_st_law<ST, LBM_LOGNH>(a, s); break;
        case LBM_NH: diag_st_law<ST, LBM_NH>(a, s); break;
        case LBM_MR: diag_st_law<ST, LBM_MR>(a, s); break;
        case LBM_YEOH: diag_st_law<ST, LBM_YEOH>(a, s); break;
        case LBM_GENT: diag_st_law<ST, LBM_GENT>(a, s); break;
        default: diag_st_law<ST, LBM_SVK>(a, s); break;
    }
}

hipError_t launch_diagnostics(const RecoverArgs& a, hipStream_t s) {
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: diag_st<LBM_F32_SHIFTED>(a, s); break;
        case LBM_F16_SHIFTED: diag_st<LBM_F16_SHIFTED>(a, s); break;
        default: diag_st<LBM_F64_PLAIN>(a, s); break;
    }
    return hipGetLastError();
}

template <int ST, int LAW>
static void init_st_law(const InitArgs& a, hipStream_t s, dim3 grid) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    if (fields) hipLaunchKernelGGL((init_pop_kernel<ST, LAW, true>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((init_pop_kernel<ST, LAW, false>), grid, dim3(kBlock), 0, s, a);
}

template <int ST>
static void init_st(const InitArgs& a, hipStream_t s, dim3 grid) {
    switch (a.cm.material) {
        case LBM_LOGNH: init_st_law<ST, LBM_LOGNH>(a, s, grid); break;
        case LBM_NH: init_st_law<ST, LBM_NH>(a, s, grid); break;
        case LBM_MR: init_st_law<ST, LBM_MR>(a, s, grid); break;
        case LBM_YEOH: init_st_law<ST, LBM_YEOH>(a, s, grid); break;
        case LBM_GENT: init_st_law<ST, LBM_GENT>(a, s, grid); break;
        default: init_st_law<ST, LBM_SVK>(a, s, grid); break;
    }
}

hipError_t launch_init_state(const InitArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(int64_t(a.cm.nx) * a.cm.ny));
    hipLaunchKernelGGL(init_state_kernel, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(int64_t(a.cm.nx) * a.cm.ny));
    hipLaunchKernelGGL(init_state_kernel, grid, dim3(kBlock), 0, s, a);
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: init_st<LBM_F32_SHIFTED>(a, s, grid); break;
        case LBM_F16_SHIFTED: init_st<LBM_F16_SHIFTED>(a, s, grid); break;
        default: init_st<LBM_F64_PLAIN>(a, s, grid); break;
    }
    return hipGetLastError();
}

}  // namespace lbm
