// Hand-written adjoint of the D2Q4 x 6 step on gfx950.
//
// The adjoint buffer holds lambda^m = dL/df^m (pre-collision populations of level m) in
// the compute type.  One adjoint step at level m, mirroring the forward step:
//   lambda*^m_q(X) = lambda^{m+1}_q(X + c_q)          (transpose of eq:streaming, a pull)
//   lambda*^m_{-d}(X0) = D lambda^{m+1}_d(X0)         (transpose of eq:boundary-general)
//   g = dL/dU^m = omega sum_q (f^eq_q)'(U^m)^T lambda*^m_q (+ probe and traction sources)
//   lambda^m_q = (1 - omega) lambda*^m_q + g           (transpose of eq:collision, eq:moment-U)
// with (f^eq_q)' from eq:feq-derivative and the Jacobian actions of eq:jacobian-actions
// through the tangent C = dP/dF (eq:stress-and-tangent), here used transposed:
//   A_X^T l = (-l3, -l5, -(l1 C_11kB + l2 C_21kB)), A_Y^T l = (-l4, -l6, -(l1 C_12kB + l2 C_22kB)).
// Parameter gradients accumulate in FP64 per node.
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"
#include "lbm_adjoint.hpp"

namespace lbm {

template <typename R>
__device__ __forceinline__ R D_sign(int bc, int k) {
    // velocity rule diag(-1,-1,1,1,1,1), traction rule diag(1,1,-1,-1,-1,-1)
    const bool vrow = k < 2;
    if (bc == LBM_VELOCITY) return vrow ? R(-1) : R(1);
    return vrow ? R(1) : R(-1);
}

template <int ST, int LAW, bool WALLS, bool FIELDS>
__global__ void __launch_bounds__(kBlock) adjoint_kernel(AdjArgs a) {
    using R = typename Storage<ST>::real;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny, ntile = cm.ntile;
    int x, y;
    if (!tile_thread(nx, ny, ntile, x, y)) return;
    const int64_t n = int64_t(nx) * ny;
    const R* __restrict__ src = (const R*)a.src;
    R* __restrict__ dst = (R*)a.dst;
    const int idx = y * nx + x;
    const int64_t own = tile_base(ntile, 24, x, y);

    // lambda*_q(X) pulls lambda_q from X + c_q: q0 from (x+1, y), q1 from (x, y+1),
    // q2 from (x-1, y), q3 from (x, y-1).  Beyond a wall the slot is the outgoing link of
    // that wall: q0 at XMAX, q1 at YMAX, q2 at XMIN, q3 at YMIN.
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    bool w0 = false, w1 = false, w2 = false, w3 = false;
    if (xp >= nx) { if (WALLS && !cm.periodic_x) { w0 = true; xp = x; } else xp = 0; }
    if (yp >= ny) { if (WALLS && !cm.periodic_y) { w1 = true; yp = y; } else yp = 0; }
    if (xm < 0) { if (WALLS && !cm.periodic_x) { w2 = true; xm = x; } else xm = nx - 1; }
    if (ym < 0) { if (WALLS && !cm.periodic_y) { w3 = true; ym = y; } else ym = ny - 1; }
    const int64_t sb[4] = {tile_base(ntile, 24, xp, y), tile_base(ntile, 24, x, yp),
                           tile_base(ntile, 24, xm, y), tile_base(ntile, 24, x, ym)};
    R l[4][6];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) l[q][k] = src[sb[q] + (6 * q + k) * kTile];
    if constexpr (WALLS) {
        // outgoing slot od of edge e takes D_e lambda_d(own node), d the missing direction
        if (w0) for (int k = 0; k < 6; ++k) l[0][k] = D_sign<R>(cm.bc[LBM_XMAX], k) * src[own + (12 + k) * kTile];
        if (w2) for (int k = 0; k < 6; ++k) l[2][k] = D_sign<R>(cm.bc[LBM_XMIN], k) * src[own + (0 + k) * kTile];
        if (w1) for (int k = 0; k < 6; ++k) l[1][k] = D_sign<R>(cm.bc[LBM_YMAX], k) * src[own + (18 + k) * kTile];
        if (w3) for (int k = 0; k < 6; ++k) l[3][k] = D_sign<R>(cm.bc[LBM_YMIN], k) * src[own + (6 + k) * kTile];
    }

    const R* rec = (const R*)a.record + tile_base(ntile, 6, x, y);
    R ft[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ft[k] = rec[(2 + k) * kTile];
    R mu, lam;
    params_at<FIELDS, R>(cm, idx, mu, lam);
    R out[4][6], inc[4];
    adj_node<R, LAW>(cm, l, ft, mu, lam, R(a.r_m), a.g_mu || a.g_lam, a.g_body != nullptr, out, inc);
    double ps[2];
    const bool probe = probe_at<R>(a, x, y, ps);
    if (probe) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            out[q][0] += R(ps[0]);
            out[q][1] += R(ps[1]);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) store_stream(dst + own + (6 * q + k) * kTile, out[q][k]);

    // parameter gradients of this level's collision.  FP64 storage adds them to the FP64
    // gradients directly; the shifted storages sum them in FP32 per block (gsum, 4 tiled
    // planes mu, lam, b1, b2) and move the block sums into the FP64 gradients at the
    // levels m with m % kGradBlock == 0 (the last adjoint step, m = 0, always folds)
    double* const g64[4] = {a.g_mu, a.g_lam, a.g_body, a.g_body ? a.g_body + n : nullptr};
    if constexpr (ST == LBM_F64_PLAIN) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (g64[j]) g64[j][idx] += double(inc[j]);
    } else if (g64[0] || g64[1] || g64[2]) {
        float* gs = (float*)a.gsum + tile_base(ntile, 4, x, y);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!g64[j]) continue;
            const float sj = gs[j * kTile] + float(inc[j]);
            if (a.fold) {
                g64[j][idx] += double(sj);
                store_stream(gs + j * kTile, 0.0f);
            } else {
                store_stream(gs + j * kTile, sj);
            }
        }
    }
    // the probe's body term (its source enters the body force's adjoint)
    if (probe && a.g_body) {
        const double hdt = 0.5 * cm.dt;
        a.g_body[idx] += a.r_m * hdt * ps[0];
        a.g_body[n + idx] += a.r_m * hdt * ps[1];
    }
}

// Traction edges, stage 1 (one thread per wall link): F^b is rebuilt from the record of
// U^m as the forward step builds it (tangential column = the wall node's own, normal
// column by the Newton solve), then dL/dF^b = lambda^{m+1}_d(X0)_F / 2 is carried through
// the solve by the implicit function theorem: with y = J^{-T} (dL/da), the tangential
// column receives -N_A y_i C_iAjB and mu, lam receive -N_A y_i dP_iA/dp.  One launch
// covers every traction edge, one wavefront per workgroup.  Each link stages
// (tbar_1, tbar_2, dL/dmu, dL/dlam) in its own slot of the staging buffer; they reach
// lambda^m and the gradients in the scatter stage, which gives a corner node the terms of
// its edges in edge order.
template <int ST, int LAW, bool FIELDS, int A>
__device__ __forceinline__ void adj_traction_solve(const AdjArgs& a, int e) {
    using R = typename Storage<ST>::real;
    const Common& cm = a.cm;
    const EdgeGeom G = edge_geom(e);
    const int L = (A == 0) ? cm.ny : cm.nx;
    constexpr int Bx = 1 - A;
    const int s = (int(blockIdx.x) - a.eblk[e]) * kTracWin + int(threadIdx.x);
    if (s >= L) return;
    const XY n0 = edge_node(G, cm.nx, cm.ny, 0, s);
    const R* rec = (const R*)a.record + tile_base(cm.ntile, 6, n0.x, n0.y);
    R tang[2], acol[2], Tv[2];
    for (int k = 0; k < 2; ++k) {
        tang[k] = rec[(2 + 2 * k + Bx) * kTile];
        acol[k] = rec[(2 + 2 * k + A) * kTile];
        Tv[k] = edge_value<R>(a.ed, e, k, s, L);
    }
    const int id0 = n0.y * cm.nx + n0.x;
    R mu, lam;
    params_at<FIELDS, R>(cm, id0, mu, lam);
    newton_column<R, LAW, true, A>(R(G.NA), tang, Tv, mu, lam, law_consts<R>(cm), acol, cm.newton_max_iter,
                                   R(cm.newton_tol));
    R f[4];
    f[A] = acol[0]; f[2 + A] = acol[1];
    f[Bx] = tang[0]; f[2 + Bx] = tang[1];
    // dL/dF^b = lambda^{m+1}_d(X0)_F / 2: from the populations, or (the second level of a
    // two-level step) from the wall line of the staging buffer
    R Fbar[4];
    if (a.lines) {
        const R* lv = (const R*)wall_lines(a.aux, cm.nx, cm.ny).lines + line_slot(cm.nx, cm.ny, e, 0, s) * 24;
        for (int k = 0; k < 4; ++k) Fbar[k] = R(0.5) * lv[6 * G.d + 2 + k];
    } else {
        const R* src = (const R*)a.src;
        const int64_t wb = tile_base(cm.ntile, 24, n0.x, n0.y);
        for (int k = 0; k < 4; ++k) Fbar[k] = R(0.5) * src[wb + (6 * G.d + 2 + k) * kTile];
    }
    R C[16];
    tangent<R, LAW, true>(f, mu, lam, law_consts<R>(cm), C);
    const R NA = R(G.NA);
    const R j00 = NA * C[4 * A + A], j01 = NA * C[4 * A + 2 + A];
    const R j10 = NA * C[8 + 4 * A + A], j11 = NA * C[8 + 4 * A + 2 + A];
    const R det = j00 * j11 - j01 * j10;
    const R ab0 = Fbar[A], ab1 = Fbar[2 + A];
    // y = J^{-T} abar
    const R y0 = (j11 * ab0 - j10 * ab1) / det;
    const R y1 = (-j01 * ab0 + j00 * ab1) / det;
    R tbar[2];
    for (int jj = 0; jj < 2; ++jj)
        tbar[jj] = Fbar[2 * jj + Bx] - NA * (y0 * C[4 * A + 2 * jj + Bx] + y1 * C[8 + 4 * A + 2 * jj + Bx]);
    R gm = R(0), gl = R(0);
    if (a.g_mu || a.g_lam) {
        R Pm[4], Pl[4];
        piola_partials<R, LAW, true>(f, law_consts<R>(cm), Pm, Pl);
        gm = -NA * (y0 * Pm[A] + y1 * Pm[2 + A]);
        gl = -NA * (y0 * Pl[A] + y1 * Pl[2 + A]);
    }
    R* aux = (R*)a.aux + 4 * (int64_t)(edge_off(cm.nx, cm.ny, e) + s);
    aux[0] = tbar[0];
    aux[1] = tbar[1];
    aux[2] = gm;
    aux[3] = gl;
}

// The edge's normal axis is a template parameter of the solve (fixed per edge, so per
// wavefront), so F, the tangent and the per-node vectors index with constants.
template <int ST, int LAW, bool FIELDS>
__global__ void __launch_bounds__(kTracWin) adj_traction_kernel(AdjArgs a) {
    int e = 0;
    while (e < 3 && int(blockIdx.x) >= a.eblk[e + 1]) ++e;
    if (e == LBM_XMIN || e == LBM_XMAX) adj_traction_solve<ST, LAW, FIELDS, 0>(a, e);
    else adj_traction_solve<ST, LAW, FIELDS, 1>(a, e);
}

// Traction edges, stage 2, for the wall node at position s of edge e: F^b's tangential
// column is that node's F of level m, so dL/dU^m there receives the staged tbar in those
// two components, for every q of lambda^m; the mu and lam terms of the link's Newton
// solve (stage 1) go to the gradients.
template <typename R, int AX>
__device__ __forceinline__ void adj_scatter_edge(const AdjArgs& a, int e, int s) {
    const Common& cm = a.cm;
    constexpr int Bx = 1 - AX;
    const R* aux = (const R*)a.aux + 4 * ((int64_t)edge_off(cm.nx, cm.ny, e) + s);
    const XY nd = edge_node(edge_geom(e), cm.nx, cm.ny, 0, s);
    const int id = nd.y * cm.nx + nd.x;
    if (a.g_mu) a.g_mu[id] += double(aux[2]);
    if (a.g_lam) a.g_lam[id] += double(aux[3]);
    R* dst = (R*)a.dst + tile_base(cm.ntile, 24, nd.x, nd.y);
    for (int q = 0; q < 4; ++q)
        for (int k = 0; k < 2; ++k) dst[(6 * q + 2 + 2 * k + Bx) * kTile] += aux[k];
}

// Stage 2 of every traction edge in one launch, one thread per wall node of each edge
// (workgroups [sblk[e], sblk[e+1]) for edge e).  A corner node lies on the wall lines of
// two traction edges; the thread of the first of them (XMIN, XMAX, YMIN, YMAX order)
// applies both edges' terms in that order and the other thread skips the node, so every
// node takes its terms in the same order as edge after edge.
template <int ST>
__global__ void __launch_bounds__(kTile) adj_traction_scatter_kernel(AdjArgs a) {
    using R = typename Storage<ST>::real;
    const Common& cm = a.cm;
    int e = 0;
    while (e < 3 && int(blockIdx.x) >= a.sblk[e + 1]) ++e;
    const int L = (e == LBM_XMIN || e == LBM_XMAX) ? cm.ny : cm.nx;
    const int s = (int(blockIdx.x) - a.sblk[e]) * kTile + int(threadIdx.x);
    if (s >= L) return;
    const XY nd = edge_node(edge_geom(e), cm.nx, cm.ny, 0, s);
    // the traction edges whose wall line holds this node: at most one along x and one
    // along y, the x edge first in edge order
    const int x = nd.x, y = nd.y;
    int ex = -1, ey = -1;
    if (cm.bc[LBM_XMIN] == LBM_TRACTION && x == 0) ex = LBM_XMIN;
    else if (cm.bc[LBM_XMAX] == LBM_TRACTION && x == cm.nx - 1) ex = LBM_XMAX;
    if (cm.bc[LBM_YMIN] == LBM_TRACTION && y == 0) ey = LBM_YMIN;
    else if (cm.bc[LBM_YMAX] == LBM_TRACTION && y == cm.ny - 1) ey = LBM_YMAX;
    if ((ex >= 0 ? ex : ey) != e) return;
    if (ex >= 0) adj_scatter_edge<R, 0>(a, ex, y);
    if (ey >= 0) adj_scatter_edge<R, 1>(a, ey, x);
}

// Probe source of the displacement loss at level m: u^N = u0 - (dt/2) v0 + dt sum_{m<N} v^m
// + (dt/2) v^N (eq:trapezoid-u), so dL/dv^m = weight * ubar with weight dt (m < N) or
// dt/2 (m = N).  One thread walks the probes in order, so repeated cells accumulate.
template <int ST>
__global__ void adj_probe_kernel(AdjArgs a) {
    using R = typename Storage<ST>::real;
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const Common& cm = a.cm;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    R* dst = (R*)a.dst;
    const double hdt = 0.5 * cm.dt;
    for (int p = 0; p < a.nprobe; ++p) {
        const int id = a.probe[p];
        if (id < 0 || int64_t(id) >= n) {
            if (cm.fault) atomicOr(cm.fault, (uint32_t)LBM_FAULT_PROBE);
            continue;
        }
        const int py = id / cm.nx, px = id - py * cm.nx;
        R* d = dst + tile_base(cm.ntile, 24, px, py);
        for (int k = 0; k < 2; ++k) {
            const double src = a.probe_weight * a.ubar[k * a.nprobe + p];
            for (int q = 0; q < 4; ++q) d[(6 * q + k) * kTile] += R(src);
            if (a.g_body) a.g_body[k * n + id] += a.r_m * hdt * src;
        }
    }
}

// ---------------------------------------------------------------- two fused adjoint levels

// Pulled adjoint populations lambda*_q(X) = lambda_q(X + c_q) of node (x, y), periodic wrap.
template <typename R>
__device__ __forceinline__ void pull_adj_node(const R* __restrict__ src, int ntile, int nx, int ny, int x, int y,
                                              R l[4][6]) {
    const int64_t b0 = tile_base(ntile, 24, wrap_inc(x, nx), y);
    const int64_t b1 = tile_base(ntile, 24, x, wrap_inc(y, ny));
    const int64_t b2 = tile_base(ntile, 24, wrap_dec(x, nx), y);
    const int64_t b3 = tile_base(ntile, 24, x, wrap_dec(y, ny));
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        l[0][k] = src[b0 + k * kTile];
        l[1][k] = src[b1 + (6 + k) * kTile];
        l[2][k] = src[b2 + (12 + k) * kTile];
        l[3][k] = src[b3 + (18 + k) * kTile];
    }
}

// The adjoint of the missing links of a wall node (transpose of eq:boundary-general): the
// slot of the outgoing direction N of each wall takes D lambda_d of the node itself, d = -N
// the missing direction (XMIN: q2 from q0, XMAX: q0 from q2, YMIN: q3 from q1, YMAX: q1 from
// q3).  `own(q, k)` gives lambda_q component k of the node.
template <typename R, typename Own>
__device__ __forceinline__ void adj_wall_slots(const Common& cm, int x, int y, Own own, R l[4][6]) {
    if (!cm.periodic_x) {
        if (x == 0)
#pragma unroll
            for (int k = 0; k < 6; ++k) l[2][k] = D_sign<R>(cm.bc[LBM_XMIN], k) * own(0, k);
        if (x == cm.nx - 1)
#pragma unroll
            for (int k = 0; k < 6; ++k) l[0][k] = D_sign<R>(cm.bc[LBM_XMAX], k) * own(2, k);
    }
    if (!cm.periodic_y) {
        if (y == 0)
#pragma unroll
            for (int k = 0; k < 6; ++k) l[3][k] = D_sign<R>(cm.bc[LBM_YMIN], k) * own(1, k);
        if (y == cm.ny - 1)
#pragma unroll
            for (int k = 0; k < 6; ++k) l[1][k] = D_sign<R>(cm.bc[LBM_YMAX], k) * own(3, k);
    }
}

// The traction edges whose wall line holds node (x, y), x edge first (edge order), or -1.
__device__ __forceinline__ void traction_edges_at(const Common& cm, int x, int y, int& ex, int& ey) {
    ex = ey = -1;
    if (!cm.periodic_x) {
        if (x == 0 && cm.bc[LBM_XMIN] == LBM_TRACTION) ex = LBM_XMIN;
        else if (x == cm.nx - 1 && cm.bc[LBM_XMAX] == LBM_TRACTION) ex = LBM_XMAX;
    }
    if (!cm.periodic_y) {
        if (y == 0 && cm.bc[LBM_YMIN] == LBM_TRACTION) ey = LBM_YMIN;
        else if (y == cm.ny - 1 && cm.bc[LBM_YMAX] == LBM_TRACTION) ey = LBM_YMAX;
    }
}

// The traction terms of a wall node at one level, as adj_traction_scatter_kernel adds them
// after a single step: lambda_q of the node takes each of its links' staged tbar in the two
// components of F^b's tangential column (F12, F22 on an x edge, F11, F21 on a y edge).
template <typename R>
__device__ __forceinline__ void add_traction_tbar(const Common& cm, const void* aux, int x, int y, R l[4][6]) {
    int ex, ey;
    traction_edges_at(cm, x, y, ex, ey);
    if (ex >= 0) {
        const R* t = (const R*)aux + 4 * (int64_t(edge_off(cm.nx, cm.ny, ex)) + y);
        const R t0 = t[0], t1 = t[1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            l[q][3] += t0;
            l[q][5] += t1;
        }
    }
    if (ey >= 0) {
        const R* t = (const R*)aux + 4 * (int64_t(edge_off(cm.nx, cm.ny, ey)) + x);
        const R t0 = t[0], t1 = t[1];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            l[q][2] += t0;
            l[q][4] += t1;
        }
    }
}

// ... and its staged mu and lam terms, into the FP64 gradients in edge order.
template <typename R>
__device__ __forceinline__ void add_traction_params(const Common& cm, const void* aux, int x, int y, double* g_mu,
                                                    double* g_lam) {
    int ex, ey;
    traction_edges_at(cm, x, y, ex, ey);
    const int64_t id = int64_t(y) * cm.nx + x;
    if (ex >= 0) {
        const R* t = (const R*)aux + 4 * (int64_t(edge_off(cm.nx, cm.ny, ex)) + y);
        if (g_mu) g_mu[id] += double(t[2]);
        if (g_lam) g_lam[id] += double(t[3]);
    }
    if (ey >= 0) {
        const R* t = (const R*)aux + 4 * (int64_t(edge_off(cm.nx, cm.ny, ey)) + x);
        if (g_mu) g_mu[id] += double(t[2]);
        if (g_lam) g_lam[id] += double(t[3]);
    }
}

// lambda^m of a node on a wall line or first interior line into the wall lines of the
// staging buffer (every such line through it; 24 values of the compute type per slot).
template <typename R>
__device__ __forceinline__ void store_adj_lines(const Common& cm, void* aux, int x, int y, const R l[4][6]) {
    const int nx = cm.nx, ny = cm.ny;
    const WallLines wl = wall_lines(aux, nx, ny);
    int er[4] = {-1, -1, -1, -1}, es[4] = {0, 0, 0, 0};
    if (!cm.periodic_x) {
        if (x <= 1) { er[LBM_XMIN] = x; es[LBM_XMIN] = y; }
        if (x >= nx - 2) { er[LBM_XMAX] = nx - 1 - x; es[LBM_XMAX] = y; }
    }
    if (!cm.periodic_y) {
        if (y <= 1) { er[LBM_YMIN] = y; es[LBM_YMIN] = x; }
        if (y >= ny - 2) { er[LBM_YMAX] = ny - 1 - y; es[LBM_YMAX] = x; }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (er[e] < 0) continue;
        R* lv = (R*)wl.lines + line_slot(nx, ny, e, er[e], es[e]) * 24;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int k = 0; k < 6; ++k) lv[6 * q + k] = l[q][k];
    }
}

// The LDS of one two-level adjoint workgroup: lambda^m of the q1 and q3 planes of every row
// wave (read by the rows below and above) and of the nodes beside the strip (q2 at c0 - 1,
// q0 at c0 + 64).
template <typename R>
struct Adj2Lds {
    R xq1[kPairWaves][6][kTile];
    R xq3[kPairWaves][6][kTile];
    R xh[2][6][kPairRows];
};

// The FP64 gradients and FP32 block sums of one node over two adjoint levels, in the order
// of two single steps: level m's increments (block sum, fold), its probe body term, the
// traction terms of level m's links at a traction wall node (tw, staged by stage 1: what
// adj_traction_scatter_kernel adds after a single step), then level m - 1's increments and
// probe body term.
template <int ST, typename R>
__device__ __forceinline__ void adj_pair_gradients(const Adj2Args& a, int x, int y, const R inc1[4], const R inc2[4],
                                                   bool probe, const double ps[2], const void* tw) {
    const Common& cm = a.cm;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    const int64_t gi = int64_t(y) * cm.nx + x;
    double* const g64[4] = {a.g_mu, a.g_lam, a.g_body, a.g_body ? a.g_body + n : nullptr};
    const double hdt = 0.5 * cm.dt;
    if constexpr (ST == LBM_F64_PLAIN) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
            if (g64[jj]) g64[jj][gi] += double(inc1[jj]);
        if (probe && a.g_body) {
            a.g_body[gi] += a.r1 * hdt * ps[0];
            a.g_body[n + gi] += a.r1 * hdt * ps[1];
        }
        if (tw) add_traction_params<R>(cm, tw, x, y, a.g_mu, a.g_lam);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
            if (g64[jj]) g64[jj][gi] += double(inc2[jj]);
        if (probe && a.g_body) {
            a.g_body[gi] += a.r2 * hdt * ps[0];
            a.g_body[n + gi] += a.r2 * hdt * ps[1];
        }
    } else {
        const bool any = g64[0] || g64[1] || g64[2];
        float* gs = (float*)a.gsum + tile_base(cm.ntile, 4, x, y);
        float sj[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        if (any) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                if (!g64[jj]) continue;
                sj[jj] = gs[jj * kTile] + float(inc1[jj]);
                if (a.fold1) {
                    g64[jj][gi] += double(sj[jj]);
                    sj[jj] = 0.0f;
                }
            }
        }
        if (probe && a.g_body) {
            a.g_body[gi] += a.r1 * hdt * ps[0];
            a.g_body[n + gi] += a.r1 * hdt * ps[1];
        }
        if (tw) add_traction_params<R>(cm, tw, x, y, a.g_mu, a.g_lam);
        if (any) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                if (!g64[jj]) continue;
                sj[jj] = sj[jj] + float(inc2[jj]);
                if (a.fold2) {
                    g64[jj][gi] += double(sj[jj]);
                    sj[jj] = 0.0f;
                }
                store_stream(gs + jj * kTile, sj[jj]);
            }
        }
        if (probe && a.g_body) {
            a.g_body[gi] += a.r2 * hdt * ps[0];
            a.g_body[n + gi] += a.r2 * hdt * ps[1];
        }
    }
}

// Two adjoint levels m and m - 1 per pass, the transpose of the two-level forward kernel: a
// workgroup owns kPairRows rows of one 64-node strip; wave w takes row y0 - 1 + w from
// lambda^{m+1} to lambda^m (with the probe source of level m), one more wave the two
// columns beside the strip, and waves 1 .. kPairRows take their row on to lambda^{m-1}.
// The adjoint pulls from X + c_q, so the rows and columns exchanged are the mirror images
// of the forward's.  Per node the arithmetic is adj_node, as in adjoint_kernel, and the
// gradient updates of the two levels (block sums, folds, the probe body term of level m)
// run in the order of two single steps, so the result is bit for bit theirs (with the
// probe table in both), the probe sources of both levels included.  WALLS: the wall slots
// of level m take the transposed wall rules and a traction wall node its staged level-m
// terms, as in adjoint_kernel followed by adj_traction_scatter_kernel; level m of the wall
// lines and first interior lines goes to the staging buffer, and the wall nodes are left
// out of the second level and of the gradients (adjoint2_wall_kernel does them).
template <int ST, int LAW, bool FIELDS, bool WALLS>
__device__ __forceinline__ void adjoint2_body(const Adj2Args& a, int strip, int blk,
                                              Adj2Lds<typename Storage<ST>::real>& sh) {
    using R = typename Storage<ST>::real;
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
    const int idx = yr * nx + xc;
    const R* __restrict__ src = (const R*)a.src;
    R* __restrict__ dst = (R*)a.dst;
    const bool gpar = a.g_mu || a.g_lam, gbody = a.g_body != nullptr;
    // a node of the grid (a lane or row beyond a wall is not; along a periodic axis every
    // lane and row is the node it wraps to)
    const bool valid = !WALLS || ((cm.periodic_x || xg < nx) && (cm.periodic_y || (r >= 0 && r < ny)));

    R l[4][6], lm[4][6], inc1[4], mu, lam;
    double ps[2] = {0.0, 0.0};
    bool probe = false;
    // the record of level m - 1 at an inner wave's node, loaded with level m + 1 so that the
    // load is in flight across the barrier (FP32 compute; in FP64 the four held values
    // would cost the kernel an occupancy step, so it loads them after the barrier)
    constexpr bool kPre = ST != LBM_F64_PLAIN;
    R ft2[4] = {R(0), R(0), R(0), R(0)};
    if (kPre && w >= 1 && w <= kPairRows) {
        const R* rec = (const R*)a.rec2 + tile_base(ntile, 6, xc, yr);
#pragma unroll
        for (int k = 0; k < 4; ++k) ft2[k] = rec[(2 + k) * kTile];
    }
    if (w < kPairWaves) {
        // lambda^{m+1} -> lambda^m on row r: q0 from x+1 and q2 from x-1 of row r (own
        // lanes shifted, the end lanes from the columns beside the strip), q1 from row r+1,
        // q3 from row r-1
        const int64_t bo = tile_base(ntile, 24, xc, yr);
        const int64_t bp = tile_base(ntile, 24, xc, wrap_near(r + 1, ny));
        const int64_t bm = tile_base(ntile, 24, xc, wrap_near(r - 1, ny));
        R own0[6], own2[6], h[6] = {};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            own0[k] = src[bo + k * kTile];
            own2[k] = src[bo + (12 + k) * kTile];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            l[1][k] = src[bp + (6 + k) * kTile];
            l[3][k] = src[bm + (18 + k) * kTile];
        }
        if (lane == 0 || lane == kTile - 1) {
            const int64_t bh = lane == kTile - 1 ? tile_base(ntile, 24, wrap_near(c0 + kTile, nx), yr)
                                                 : tile_base(ntile, 24, wrap_near(c0 - 1, nx), yr) + 12 * kTile;
#pragma unroll
            for (int k = 0; k < 6; ++k) h[k] = src[bh + k * kTile];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const R dn = __shfl_down(own0[k], 1), up = __shfl_up(own2[k], 1);
            l[0][k] = lane == kTile - 1 ? h[k] : dn;
            l[2][k] = lane == 0 ? h[k] : up;
        }
        // (a valid node's unwrapped position equals its wrapped one along every wall axis,
        // and the wrapped one is the node along a periodic axis: the wall code takes xc, yr)
        if constexpr (WALLS) {
            if (valid) {
                const R* on = src + bo;
                adj_wall_slots<R>(cm, xc, yr, [&](int q, int k) {
                    return q == 0 ? own0[k] : q == 2 ? own2[k] : on[(6 * q + k) * kTile];
                }, l);
            }
        }
        const R* rec = (const R*)a.rec1 + tile_base(ntile, 6, xc, yr);
        R ft[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) ft[k] = rec[(2 + k) * kTile];
        params_at<FIELDS, R>(cm, idx, mu, lam);
        adj_node<R, LAW>(cm, l, ft, mu, lam, R(a.r1), gpar, gbody, lm, inc1);
        probe = probe_at<R>(a, xc, yr, ps);
        if (probe) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lm[q][0] += R(ps[0]);
                lm[q][1] += R(ps[1]);
            }
        }
        if constexpr (WALLS) {
            if (valid) {
                add_traction_tbar<R>(cm, a.aux, xc, yr, lm);
                store_adj_lines<R>(cm, a.aux, xc, yr, lm);
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            xq1[w][k][lane] = lm[1][k];
            xq3[w][k][lane] = lm[3][k];
            l[0][k] = __shfl_down(lm[0][k], 1);
            l[2][k] = __shfl_up(lm[2][k], 1);
        }
    } else {
        // the nodes beside the strip: lane j < kPairRows at (c0 - 1, y0 + j), lane
        // kPairRows + j at (c0 + 64, y0 + j); the other lanes repeat the last node
        const int j = min(lane, 2 * kPairRows - 1);
        const int side = j / kPairRows, row = j - side * kPairRows;
        const int hx = wrap_near(side == 0 ? c0 - 1 : c0 + kTile, nx), hy = wrap_near(y0 + row, ny);
        R lh[4][6], oh[4][6], ih[4], muh, lamh, fth[4];
        pull_adj_node<R>(src, ntile, nx, ny, hx, hy, lh);
        bool hvalid = true;
        if constexpr (WALLS) {
            const int hxg = side == 0 ? c0 - 1 : c0 + kTile, hyg = y0 + row;
            hvalid = (cm.periodic_x || (hxg >= 0 && hxg < nx)) && (cm.periodic_y || hyg < ny);
            if (hvalid) {
                const R* hown = src + tile_base(ntile, 24, hx, hy);
                adj_wall_slots<R>(cm, hx, hy, [&](int q, int k) { return hown[(6 * q + k) * kTile]; }, lh);
            }
        }
        const R* rec = (const R*)a.rec1 + tile_base(ntile, 6, hx, hy);
#pragma unroll
        for (int k = 0; k < 4; ++k) fth[k] = rec[(2 + k) * kTile];
        params_at<FIELDS, R>(cm, hy * nx + hx, muh, lamh);
        adj_node<R, LAW>(cm, lh, fth, muh, lamh, R(a.r1), false, false, oh, ih);
        double hs[2];
        if (probe_at<R>(a, hx, hy, hs)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                oh[q][0] += R(hs[0]);
                oh[q][1] += R(hs[1]);
            }
        }
        if constexpr (WALLS) {
            if (hvalid) add_traction_tbar<R>(cm, a.aux, hx, hy, oh);
        }
        if (lane < 2 * kPairRows) {
#pragma unroll
            for (int k = 0; k < 6; ++k) xh[side][k][row] = side == 0 ? oh[2][k] : oh[0][k];
        }
    }
    __syncthreads();

    // lambda^m -> lambda^{m-1} on row r for the inner waves
    const int xo = c0 + lane;
    if (w >= 1 && w <= kPairRows) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            l[1][k] = xq1[w + 1][k][lane];
            l[3][k] = xq3[w - 1][k][lane];
            // selected by value, as in the forward two-level kernel
            const R e0 = xh[1][k][w - 1], e2 = xh[0][k][w - 1];
            l[0][k] = lane == kTile - 1 ? e0 : l[0][k];
            l[2][k] = lane == 0 ? e2 : l[2][k];
        }
        if constexpr (!kPre) {
            const R* rec = (const R*)a.rec2 + tile_base(ntile, 6, xc, yr);
#pragma unroll
            for (int k = 0; k < 4; ++k) ft2[k] = rec[(2 + k) * kTile];
        }
        R out[4][6], inc2[4];
        adj_node<R, LAW>(cm, l, ft2, mu, lam, R(a.r2), gpar, gbody, out, inc2);
        if (probe) {
            // the probe source of level m - 1 (same node, same weight as level m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                out[q][0] += R(ps[0]);
                out[q][1] += R(ps[1]);
            }
        }
        const bool wall_node = WALLS && ((!cm.periodic_x && (xo == 0 || xo == nx - 1)) ||
                                         (!cm.periodic_y && (r == 0 || r == ny - 1)));
        if (r < ny && xo < nx && !wall_node) {
            const int64_t ob = tile_base(ntile, 24, xo, r);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < 6; ++k) store_stream(dst + ob + (6 * q + k) * kTile, out[q][k]);
            adj_pair_gradients<ST>(a, xo, r, inc1, inc2, probe, ps, nullptr);
        }
    }
}

template <int ST, int LAW, bool FIELDS, bool WALLS>
__global__ void __launch_bounds__((kPairWaves + 1) * kTile) adjoint2_kernel(Adj2Args a) {
    __shared__ Adj2Lds<typename Storage<ST>::real> sh;
    int strip, blk;
    pair_block(a.map, remap_tile(blockIdx.x, gridDim.x), strip, blk);
    adjoint2_body<ST, LAW, FIELDS, WALLS>(a, strip, blk, sh);
}

// The wall nodes of a two-level adjoint step on a grid with walls, one thread per link slot
// of the staging buffer (a corner node is taken by the first of its edges): level m as the
// bulk pass computes it (pulled from lambda^{m+1} in HBM), level m - 1 from the wall lines
// of lambda^m that the bulk pass staged, and both levels' gradient updates in the order of
// two single steps.  The traction terms of level m - 1 come after this kernel, from stage 1
// on the staged lines and the scatter, as after a single step.
template <int ST, int LAW, bool FIELDS>
__global__ void __launch_bounds__(kTile) adjoint2_wall_kernel(Adj2Args a) {
    using R = typename Storage<ST>::real;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny;
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
    const int ntile = cm.ntile;
    const R* src = (const R*)a.src;
    const int idx = y * nx + x;
    const bool gpar = a.g_mu || a.g_lam, gbody = a.g_body != nullptr;
    // the wall beyond which the pull of direction q would reach: q0 pulls from x+1 (XMAX),
    // q1 from y+1 (YMAX), q2 from x-1 (XMIN), q3 from y-1 (YMIN)
    const bool beyond[4] = {on[LBM_XMAX], on[LBM_YMAX], on[LBM_XMIN], on[LBM_YMIN]};

    // level m
    R l[4][6], lm[4][6], inc1[4], mu, lam;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (beyond[q]) continue;
        const int sx = wrap_index(x + dir_i(q), nx), sy = wrap_index(y + dir_j(q), ny);
        const R* sp = src + tile_base(ntile, 24, sx, sy);
#pragma unroll
        for (int k = 0; k < 6; ++k) l[q][k] = sp[(6 * q + k) * kTile];
    }
    {
        const R* on_ = src + tile_base(ntile, 24, x, y);
        adj_wall_slots<R>(cm, x, y, [&](int q, int k) { return on_[(6 * q + k) * kTile]; }, l);
    }
    const R* rec1 = (const R*)a.rec1 + tile_base(ntile, 6, x, y);
    R ft[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) ft[k] = rec1[(2 + k) * kTile];
    params_at<FIELDS, R>(cm, idx, mu, lam);
    adj_node<R, LAW>(cm, l, ft, mu, lam, R(a.r1), gpar, gbody, lm, inc1);
    double ps[2] = {0.0, 0.0};
    const bool probe = probe_at<R>(a, x, y, ps);
    if (probe) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            lm[q][0] += R(ps[0]);
            lm[q][1] += R(ps[1]);
        }
    }
    add_traction_tbar<R>(cm, a.aux, x, y, lm);

    // level m - 1: lambda^m of the neighbours from the wall lines, of the node itself from lm
    const WallLines wl = wall_lines(a.aux, nx, ny);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (beyond[q]) continue;
        const int sx = wrap_index(x + dir_i(q), nx), sy = wrap_index(y + dir_j(q), ny);
        int le = 0, lr = 0, ls = 0;
        find_line(cm, sx, sy, le, lr, ls);
        const R* sp = (const R*)wl.lines + line_slot(nx, ny, le, lr, ls) * 24;
#pragma unroll
        for (int k = 0; k < 6; ++k) l[q][k] = sp[6 * q + k];
    }
    adj_wall_slots<R>(cm, x, y, [&](int q, int k) { return lm[q][k]; }, l);
    const R* rec2 = (const R*)a.rec2 + tile_base(ntile, 6, x, y);
#pragma unroll
    for (int k = 0; k < 4; ++k) ft[k] = rec2[(2 + k) * kTile];
    R out[4][6], inc2[4];
    adj_node<R, LAW>(cm, l, ft, mu, lam, R(a.r2), gpar, gbody, out, inc2);
    if (probe) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            out[q][0] += R(ps[0]);
            out[q][1] += R(ps[1]);
        }
    }
    R* dst = (R*)a.dst + tile_base(ntile, 24, x, y);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) store_stream(dst + (6 * q + k) * kTile, out[q][k]);
    adj_pair_gradients<ST>(a, x, y, inc1, inc2, probe, ps, a.aux);
}

// The probe table: bit x mod 64 of word (y, x / 64) marks a probe, field holds the sum of
// the ubar of the probes on that cell (2 planes).  One thread walks the probes in order (the
// buffers are cleared by adj_probe_clear_kernel first).
__global__ void adj_probe_clear_kernel(uint64_t* mask, int64_t nmask, double* field, int64_t nfield) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nmask) mask[i] = 0ull;
    if (i < nfield) field[i] = 0.0;
}

__global__ void adj_probe_table_kernel(Common cm, const int32_t* probe, const double* ubar, int nprobe,
                                       uint64_t* mask, double* field) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    for (int p = 0; p < nprobe; ++p) {
        const int id = probe[p];
        if (id < 0 || int64_t(id) >= n) {
            if (cm.fault) atomicOr(cm.fault, (uint32_t)LBM_FAULT_PROBE);
            continue;
        }
        const int py = id / cm.nx, px = id - py * cm.nx;
        mask[int64_t(py) * cm.ntile + (px >> 6)] |= 1ull << (px & 63);
        field[id] += ubar[p];
        field[n + id] += ubar[nprobe + p];
    }
}

// ---------------------------------------------------------------- adjoint of the init

// Per node: the transposes of eq:init-expanded, eq:init-deltaPq and eq:init-Zq-components
// (F0 held fixed).  Writes the seeds (dL/dv0 direct, dL/d(d_X v0), dL/d(d_Y v0)) as
// scratch planes 6..11 and adds the parameter and body parts.
template <int ST, int LAW, bool FIELDS>
__global__ void __launch_bounds__(kBlock) adj_init_kernel(AdjInitArgs a) {
    using R = typename Storage<ST>::real;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny;
    const int64_t n = int64_t(nx) * ny;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = int(idx / nx), x = int(idx - int64_t(y) * nx);
    double* scr = (double*)a.scratch;
    const double c = cm.c, hdt = 0.5 * cm.dt;
    const double inv2h = 1.0 / (2.0 * cm.dx);
    double U0[6], dX[6], dY[6];
    for (int k = 0; k < 6; ++k) {
        const double* pl = scr + k * n;
        U0[k] = pl[idx];
        dX[k] = fd_along<double>([&](int s) { return pl[int64_t(y) * nx + s]; }, x, nx, cm.periodic_x, inv2h);
        dY[k] = fd_along<double>([&](int s) { return pl[int64_t(s) * nx + x]; }, y, ny, cm.periodic_y, inv2h);
    }
    double mu, lam;
    params_at<FIELDS, double>(cm, (int)idx, mu, lam);
    // The actions on a 2 x 2 array Z (flat index 2i + A) of the tangent C = dP/dF and of
    // its parts Cm = dC/dmu, Cl = dC/dlam (each symmetric in iA <-> kB).  For log-NH and NH,
    // C_iAkB = mu d_ik d_AB + a H_iB H_kA + b H_iA H_kB, whose action is
    // mu Z + a H Z^T H + b tr(H^T Z) H, so no 4 x 4 array is formed (the three arrays would
    // hold 96 registers); the other laws form them from their forward-mode tangent.
    constexpr bool lame = LAW == LBM_LOGNH || LAW == LBM_NH;
    double C[16], Cm[16], Cl[16], Pm[4], Pl[4];
    Kin<double> kk;
    double aC = 0.0, bC = 0.0, aL = 0.0, bL = 0.0;
    if constexpr (lame) {
        kk = kinematics<double, true>(&U0[2]);
        if constexpr (LAW == LBM_LOGNH) {
            aC = mu - lam * kk.L;
            bC = lam;
            aL = -kk.L;
            bL = 1.0;
        } else {
            aC = mu - 0.5 * lam * kk.Jsq_m1;
            bC = lam * kk.J * kk.J;
            aL = -0.5 * kk.Jsq_m1;
            bL = kk.J * kk.J;
        }
        const double v = LAW == LBM_LOGNH ? kk.L : 0.5 * kk.Jsq_m1;
        for (int k = 0; k < 4; ++k) {
            Pm[k] = kk.FmH[k];
            Pl[k] = v * kk.H[k];
        }
    } else {
        tangent<double, LAW, true>(&U0[2], mu, lam, law_consts<double>(cm), C);
        tangent<double, LAW, true>(&U0[2], 1.0, 0.0, law_consts<double>(cm), Cm);
        tangent<double, LAW, true>(&U0[2], 0.0, 1.0, law_consts<double>(cm), Cl);
        piola_partials<double, LAW, true>(&U0[2], law_consts<double>(cm), Pm, Pl);
    }
    // which: 0 C, 1 Cm, 2 Cl
    auto act = [&](int which, const double Z[4], double out[4]) {
        if constexpr (lame) {
            const double* H = kk.H;
            const double m = which == 0 ? mu : which == 1 ? 1.0 : 0.0;
            const double a2 = which == 0 ? aC : which == 1 ? 1.0 : aL;
            const double b2 = which == 0 ? bC : which == 1 ? 0.0 : bL;
            const double tr = H[0] * Z[0] + H[1] * Z[1] + H[2] * Z[2] + H[3] * Z[3];
            for (int i = 0; i < 2; ++i)
                for (int A = 0; A < 2; ++A) {
                    double hz = 0.0;
                    for (int B = 0; B < 2; ++B)
                        hz += H[2 * i + B] * (Z[B] * H[A] + Z[2 + B] * H[2 + A]);
                    out[2 * i + A] = m * Z[2 * i + A] + a2 * hz + b2 * tr * H[2 * i + A];
                }
        } else if (which == 0) {
            // the transposed action sum_iA C_iAkB Z_iA (the forward-mode C is symmetric only
            // up to rounding)
            for (int kB = 0; kB < 4; ++kB) {
                double acc = 0.0;
                for (int iA = 0; iA < 4; ++iA) acc += C[4 * iA + kB] * Z[iA];
                out[kB] = acc;
            }
        } else {
            const double* T = which == 1 ? Cm : Cl;
            for (int iA = 0; iA < 4; ++iA) {
                double acc = 0.0;
                for (int kB = 0; kB < 4; ++kB) acc += T[4 * iA + kB] * Z[kB];
                out[iA] = acc;
            }
        }
    };
    const R* l0 = (const R*)a.lam0;
    double vb[2] = {0, 0}, vXb[2] = {0, 0}, vYb[2] = {0, 0}, Bb[2] = {0, 0};
    double dPXb[4] = {0, 0, 0, 0}, dPYb[4] = {0, 0, 0, 0};
    double gmu = 0.0, glam = 0.0;
    for (int q = 0; q < 4; ++q) {
        const double i = dir_i(q), j = dir_j(q);
        double ell[6];
        for (int k = 0; k < 6; ++k) ell[k] = double(l0[tile_base(cm.ntile, 24, x, y) + (6 * q + k) * kTile]);
        // equilibrium part f^eq_q(U0)
        vb[0] += 0.25 * (ell[0] - (2.0 / c) * (i * ell[2] + j * ell[3]));
        vb[1] += 0.25 * (ell[1] - (2.0 / c) * (i * ell[4] + j * ell[5]));
        gmu += (0.5 / c) * -(i * (ell[0] * Pm[0] + ell[1] * Pm[2]) + j * (ell[0] * Pm[1] + ell[1] * Pm[3]));
        glam += (0.5 / c) * -(i * (ell[0] * Pl[0] + ell[1] * Pl[2]) + j * (ell[0] * Pl[1] + ell[1] * Pl[3]));
        // correction part -(dt/2) D_q f^eq
        double w[6];
        for (int k = 0; k < 6; ++k) w[k] = -hdt * ell[k];
        const double Z1b = 0.25 * (w[0] - (2.0 * i / c) * w[2] - (2.0 * j / c) * w[3]);
        const double Z2b = 0.25 * (w[1] - (2.0 * i / c) * w[4] - (2.0 * j / c) * w[5]);
        const double dPb[4] = {-(0.5 / c) * i * w[0], -(0.5 / c) * j * w[0], -(0.5 / c) * i * w[1],
                               -(0.5 / c) * j * w[1]};
        double ZF[4];
        ZF[0] = dX[0] + c * (i * dX[2] + j * dY[2]);
        ZF[1] = dY[0] + c * (i * dX[3] + j * dY[3]);
        ZF[2] = dX[1] + c * (i * dX[4] + j * dY[4]);
        ZF[3] = dY[1] + c * (i * dX[5] + j * dY[5]);
        double ZFb[4], CdP[4], CmZ[4], ClZ[4];
        act(0, dPb, CdP);                         // sum_iA C_iAkB dPb_iA
        for (int kB = 0; kB < 4; ++kB) ZFb[kB] = 0.25 * w[2 + kB] + CdP[kB];
        act(1, ZF, CmZ);
        act(2, ZF, ClZ);
        for (int iA = 0; iA < 4; ++iA) {
            gmu += dPb[iA] * CmZ[iA];
            glam += dPb[iA] * ClZ[iA];
        }
        Bb[0] += Z1b;
        Bb[1] += Z2b;
        dPXb[0] += Z1b;
        dPYb[1] += Z1b;
        dPXb[2] += Z2b;
        dPYb[3] += Z2b;
        vXb[0] += c * i * Z1b + ZFb[0];
        vYb[0] += c * j * Z1b + ZFb[1];
        vXb[1] += c * i * Z2b + ZFb[2];
        vYb[1] += c * j * Z2b + ZFb[3];
    }
    {
        double CmX[4], CmY[4], ClX[4], ClY[4];
        act(1, &dX[2], CmX);
        act(1, &dY[2], CmY);
        act(2, &dX[2], ClX);
        act(2, &dY[2], ClY);
        for (int iA = 0; iA < 4; ++iA) {
            gmu += dPXb[iA] * CmX[iA] + dPYb[iA] * CmY[iA];
            glam += dPXb[iA] * ClX[iA] + dPYb[iA] * ClY[iA];
        }
    }
    if (a.g_mu) a.g_mu[idx] += gmu;
    if (a.g_lam) a.g_lam[idx] += glam;
    if (a.g_body) {
        a.g_body[idx] += a.r0 * Bb[0];
        a.g_body[n + idx] += a.r0 * Bb[1];
    }
    scr[6 * n + idx] = vb[0];
    scr[7 * n + idx] = vb[1];
    scr[8 * n + idx] = vXb[0];
    scr[9 * n + idx] = vXb[1];
    scr[10 * n + idx] = vYb[0];
    scr[11 * n + idx] = vYb[1];
}

// dL/dv0 = direct seed + (finite-difference operators)^T applied to the gradient seeds.
__global__ void __launch_bounds__(kBlock) adj_init_gather_kernel(AdjInitArgs a) {
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny;
    const int64_t n = int64_t(nx) * ny;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int y = int(idx / nx), x = int(idx - int64_t(y) * nx);
    const double* scr = (const double*)a.scratch;
    const double inv2h = 1.0 / (2.0 * cm.dx);
    for (int k = 0; k < 2; ++k) {
        const double* pX = scr + (8 + k) * n;
        const double* pY = scr + (10 + k) * n;
        double v = scr[(6 + k) * n + idx];
        v += fd_along_T<double>([&](int s) { return pX[int64_t(y) * nx + s]; }, x, nx, cm.periodic_x, inv2h);
        v += fd_along_T<double>([&](int s) { return pY[int64_t(s) * nx + x]; }, y, ny, cm.periodic_y, inv2h);
        a.g_v0[k * n + idx] = v;
    }
}

// u*^0 = u0 - (dt/2) v0 contributes -(dt/2) ubar at the probes.
__global__ void adj_init_probe_kernel(AdjInitArgs a) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t n = int64_t(a.cm.nx) * a.cm.ny;
    const double hdt = 0.5 * a.cm.dt;
    for (int p = 0; p < a.nprobe; ++p) {
        const int id = a.probe[p];
        if (id < 0 || int64_t(id) >= n) {
            if (a.cm.fault) atomicOr(a.cm.fault, (uint32_t)LBM_FAULT_PROBE);
            continue;
        }
        for (int k = 0; k < 2; ++k) a.g_v0[k * n + id] -= hdt * a.ubar[k * a.nprobe + p];
    }
}

// ---------------------------------------------------------------- dispatch

static inline unsigned nblk(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

template <int ST, int LAW>
static hipError_t adjoint_st_law(const AdjArgs& a0, hipStream_t s) {
    AdjArgs a = a0;
    const bool walls = !(a.cm.periodic_x && a.cm.periodic_y);
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    // stage 1 of every traction edge (one launch) reads lambda^{m+1} before the bulk kernel
    // writes lambda^m; each edge stages its values in its own slice of aux
    a.eblk[0] = 0;
    for (int e = 0; e < 4; ++e) {
        const int L = (e == LBM_XMIN || e == LBM_XMAX) ? a.cm.ny : a.cm.nx;
        a.eblk[e + 1] = a.eblk[e] + (a.cm.bc[e] == LBM_TRACTION ? (L + kTracWin - 1) / kTracWin : 0);
    }
    if (a.eblk[4] > 0) {
        if (fields) hipLaunchKernelGGL((adj_traction_kernel<ST, LAW, true>), dim3(a.eblk[4]), dim3(kTracWin), 0, s, a);
        else hipLaunchKernelGGL((adj_traction_kernel<ST, LAW, false>), dim3(a.eblk[4]), dim3(kTracWin), 0, s, a);
    }
    const dim3 grid(unsigned((int64_t(a.cm.ntile) * a.cm.ny + kTilesPerBlock - 1) / kTilesPerBlock));
    const dim3 block(kTile * kTilesPerBlock);
    if (walls) {
        if (fields) hipLaunchKernelGGL((adjoint_kernel<ST, LAW, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((adjoint_kernel<ST, LAW, true, false>), grid, block, 0, s, a);
    } else {
        if (fields) hipLaunchKernelGGL((adjoint_kernel<ST, LAW, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((adjoint_kernel<ST, LAW, false, false>), grid, block, 0, s, a);
    }
    // stage 2 of every traction edge, one launch (nodes two edges share go to the first)
    a.sblk[0] = 0;
    for (int e = 0; e < 4; ++e) {
        const int L = (e == LBM_XMIN || e == LBM_XMAX) ? a.cm.ny : a.cm.nx;
        a.sblk[e + 1] = a.sblk[e] + (a.cm.bc[e] == LBM_TRACTION ? (L + kTile - 1) / kTile : 0);
    }
    if (a.sblk[4] > 0) hipLaunchKernelGGL((adj_traction_scatter_kernel<ST>), dim3(a.sblk[4]), dim3(kTile), 0, s, a);
    // without a probe table the probe sources are added by one thread walking the probes
    if (!a.pmask && a.nprobe > 0 && a.probe_weight != 0.0)
        hipLaunchKernelGGL((adj_probe_kernel<ST>), dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int ST>
static hipError_t adjoint_st(const AdjArgs& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: return adjoint_st_law<ST, LBM_LOGNH>(a, s);
        case LBM_NH: return adjoint_st_law<ST, LBM_NH>(a, s);
        case LBM_MR: return adjoint_st_law<ST, LBM_MR>(a, s);
        case LBM_YEOH: return adjoint_st_law<ST, LBM_YEOH>(a, s);
        case LBM_GENT: return adjoint_st_law<ST, LBM_GENT>(a, s);
        default: return adjoint_st_law<ST, LBM_SVK>(a, s);
    }
}

hipError_t launch_adjoint(const AdjArgs& a, hipStream_t s) {
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: return adjoint_st<LBM_F32_SHIFTED>(a, s);
        case LBM_F16_SHIFTED: return adjoint_st<LBM_F16_SHIFTED>(a, s);
        default: return adjoint_st<LBM_F64_PLAIN>(a, s);
    }
}

template <int ST, int LAW>
static void adj_init_st_law(const AdjInitArgs& a, hipStream_t s, dim3 grid) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    if (fields) hipLaunchKernelGGL((adj_init_kernel<ST, LAW, true>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((adj_init_kernel<ST, LAW, false>), grid, dim3(kBlock), 0, s, a);
}

template <int ST>
static void adj_init_st(const AdjInitArgs& a, hipStream_t s, dim3 grid) {
    switch (a.cm.material) {
        case LBM_LOGNH: adj_init_st_law<ST, LBM_LOGNH>(a, s, grid); break;
        case LBM_NH: adj_init_st_law<ST, LBM_NH>(a, s, grid); break;
        case LBM_MR: adj_init_st_law<ST, LBM_MR>(a, s, grid); break;
        case LBM_YEOH: adj_init_st_law<ST, LBM_YEOH>(a, s, grid); break;
        case LBM_GENT: adj_init_st_law<ST, LBM_GENT>(a, s, grid); break;
        default: adj_init_st_law<ST, LBM_SVK>(a, s, grid); break;
    }
}

// The traction stages of the adjoint at one level (AdjArgs of a two-level step): stage 1
// reads lambda of the level above from `src` or, with `lines`, from the staged wall lines.
static AdjArgs traction_args(const Adj2Args& a2, const void* record, const EdgeData& ed, int lines) {
    AdjArgs a{};
    a.cm = a2.cm;
    a.src = a2.src;
    a.dst = a2.dst;
    a.record = record;
    a.g_mu = a2.g_mu;
    a.g_lam = a2.g_lam;
    a.aux = a2.aux;
    a.ed = ed;
    a.lines = lines;
    a.eblk[0] = a.sblk[0] = 0;
    for (int e = 0; e < 4; ++e) {
        const int L = (e == LBM_XMIN || e == LBM_XMAX) ? a.cm.ny : a.cm.nx;
        const bool tr = a.cm.bc[e] == LBM_TRACTION;
        a.eblk[e + 1] = a.eblk[e] + (tr ? (L + kTracWin - 1) / kTracWin : 0);
        a.sblk[e + 1] = a.sblk[e] + (tr ? (L + kTile - 1) / kTile : 0);
    }
    return a;
}

template <int ST, int LAW, bool FIELDS>
static void adj_traction_stage1(const AdjArgs& a, hipStream_t s) {
    if (a.eblk[4] > 0) hipLaunchKernelGGL((adj_traction_kernel<ST, LAW, FIELDS>), dim3(a.eblk[4]), dim3(kTracWin), 0, s, a);
}

template <int ST, int LAW, bool FIELDS>
static void adjoint2_launch(const Adj2Args& a0, hipStream_t s) {
    const dim3 block((kPairWaves + 1) * kTile);
    const int nstrip = a0.nstrip, nblk = (a0.cm.ny + kPairRows - 1) / kPairRows;
    auto go = [&](const PairMap& m, bool w) {
        const int64_t nb = pair_map_blocks(m);
        if (nb <= 0) return;
        Adj2Args a = a0;
        a.map = m;
        if (w) hipLaunchKernelGGL((adjoint2_kernel<ST, LAW, FIELDS, true>), dim3(unsigned(nb)), block, 0, s, a);
        else hipLaunchKernelGGL((adjoint2_kernel<ST, LAW, FIELDS, false>), dim3(unsigned(nb)), block, 0, s, a);
    };
    const bool walls = !(a0.cm.periodic_x && a0.cm.periodic_y);
    if (!walls) {
        go(pair_map(nstrip, nblk, 0, nstrip, 0, nblk), false);
        return;
    }
    // stage 1 of level m's traction links, from lambda^{m+1}
    adj_traction_stage1<ST, LAW, FIELDS>(traction_args(a0, a0.rec1, a0.ed1, 0), s);
    // the bulk: the blocks whose level-m region (columns c0 - 1 .. c0 + 64, rows y0 - 1 ..
    // y0 + kPairRows) keeps two nodes away from every wall run the periodic code, the
    // blocks along the walls the wall code (the same split as the two-level forward)
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
    } else {
        const PairMap inner = pair_map(nstrip, nblk, s_lo, s_hi, b_lo, b_hi);
        PairMap rim = inner;
        rim.mode = 1;
        go(inner, false);
        go(rim, true);
    }
    // the wall nodes over both levels (one wavefront per workgroup: latency-bound)
    const int links = 2 * a0.cm.nx + 2 * a0.cm.ny;
    hipLaunchKernelGGL((adjoint2_wall_kernel<ST, LAW, FIELDS>), dim3(unsigned((links + kTile - 1) / kTile)),
                       dim3(kTile), 0, s, a0);
    // level m - 1's traction links: stage 1 from the staged wall lines of lambda^m, then the
    // scatter into lambda^{m-1} and the gradients
    const AdjArgs t2 = traction_args(a0, a0.rec2, a0.ed2, 1);
    adj_traction_stage1<ST, LAW, FIELDS>(t2, s);
    if (t2.sblk[4] > 0) hipLaunchKernelGGL((adj_traction_scatter_kernel<ST>), dim3(t2.sblk[4]), dim3(kTile), 0, s, t2);
}

template <int ST, int LAW>
static hipError_t adjoint2_st_law(const Adj2Args& a, hipStream_t s) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    if (fields) adjoint2_launch<ST, LAW, true>(a, s);
    else adjoint2_launch<ST, LAW, false>(a, s);
    return hipGetLastError();
}

template <int ST>
static hipError_t adjoint2_st(const Adj2Args& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: return adjoint2_st_law<ST, LBM_LOGNH>(a, s);
        case LBM_NH: return adjoint2_st_law<ST, LBM_NH>(a, s);
        case LBM_MR: return adjoint2_st_law<ST, LBM_MR>(a, s);
        case LBM_YEOH: return adjoint2_st_law<ST, LBM_YEOH>(a, s);
        case LBM_GENT: return adjoint2_st_law<ST, LBM_GENT>(a, s);
        default: return adjoint2_st_law<ST, LBM_SVK>(a, s);
    }
}

hipError_t launch_adjoint2(const Adj2Args& a, hipStream_t s) {
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: return adjoint2_st<LBM_F32_SHIFTED>(a, s);
        case LBM_F16_SHIFTED: return adjoint2_st<LBM_F16_SHIFTED>(a, s);
        default: return adjoint2_st<LBM_F64_PLAIN>(a, s);
    }
}

hipError_t launch_probe_table(const Common& cm, const int32_t* probe, const double* ubar, int nprobe,
                              uint64_t* mask, double* field, hipStream_t s) {
    const int64_t nmask = int64_t(cm.ntile) * cm.ny, nfield = 2 * int64_t(cm.nx) * cm.ny;
    const int64_t m = nmask > nfield ? nmask : nfield;
    hipLaunchKernelGGL(adj_probe_clear_kernel, dim3(nblk(m)), dim3(kBlock), 0, s, mask, nmask, field, nfield);
    if (nprobe > 0)
        hipLaunchKernelGGL(adj_probe_table_kernel, dim3(1), dim3(64), 0, s, cm, probe, ubar, nprobe, mask, field);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(const AdjInitArgs& a, hipStream_t s) {
    const dim3 grid(nblk(int64_t(a.cm.nx) * a.cm.ny));
    // U0 = (v0, grad u0) into scratch planes 0..5, as lbm_init builds it
    InitArgs ia{};
    ia.cm = a.cm;
    ia.v0 = a.v0;
    ia.u0 = a.u0;
    for (int k = 0; k < 4; ++k) ia.Fbar[k] = a.Fbar[k];
    ia.r0 = a.r0;
    ia.scratch = a.scratch;
    hipError_t err = launch_init_state(ia, s);
    if (err != hipSuccess) return err;
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: adj_init_st<LBM_F32_SHIFTED>(a, s, grid); break;
        case LBM_F16_SHIFTED: adj_init_st<LBM_F16_SHIFTED>(a, s, grid); break;
        default: adj_init_st<LBM_F64_PLAIN>(a, s, grid); break;
    }
    hipLaunchKernelGGL(adj_init_gather_kernel, grid, dim3(kBlock), 0, s, a);
    if (a.nprobe > 0) hipLaunchKernelGGL(adj_init_probe_kernel, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace lbm
