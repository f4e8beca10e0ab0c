// Forward kernels of the D2Q4 x 6 vectorial LBM on gfx950: the fused collide-stream step
// (Sec. 3.7), the traction-wall F^b solve (Sec. 3.6), the second-order initialisation
// (Sec. 3.4) and the recoveries from stored post-collision populations (Sec. 3.5).  The
// per-node update is in lbm_collide.hpp, the two-level kernels in lbm_pair.hip.
//
// Layout: populations, u* and records in 64-node row tiles holding all their planes
// contiguously (tile_base in lbm_device.hpp).  One thread per node, one wavefront per
// tile, kTilesPerBlock tiles per workgroup; the tile order is remapped so that each of the
// eight XCDs sweeps a contiguous band of rows (its L2 then serves the one-element overlap
// of the x -/+ 1 pulls between adjacent tiles).  Each stored value is written once per
// pass, with non-temporal stores.
#include <algorithm>

#include "lbm_collide.hpp"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"

namespace lbm {

// F^b of every link of the traction edges at step n -> n+1 (Sec. 3.6).  Reading of the
// interior values the paper takes F^b's tangential column from: the wall node's own F of
// level n (recovered from its stored populations); the Newton solve of the traction
// equations starts from that node's normal column.
//
// One launch covers every traction edge (each edge reads level n only and writes its own
// slice of the staging buffer), one wavefront per workgroup and one lane per link: the
// solve is latency-bound, so the links are spread over as many compute units as there are
// wavefronts.  The edge's normal axis AX is a template parameter (fixed per edge, so per
// wavefront): with the axis known, F, the tangent and the per-node vectors index with
// constants and stay in registers.
template <int ST, int LAW, bool FIELDS, bool LINES, int AX>
__device__ __forceinline__ void traction_solve(const TractionArgs& a, int e) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    const Common& cm = a.cm;
    const EdgeGeom G = edge_geom(e);
    const int L = (AX == 0) ? cm.ny : cm.nx;
    constexpr int Bx = 1 - AX;
    const int s = (int(blockIdx.x) - a.eblk[e]) * kTracWin + int(threadIdx.x);
    if (s >= L) return;
    const int64_t n = int64_t(cm.nx) * cm.ny;
    const R hdt = R(0.5 * cm.dt);

    // U of level n at the wall node
    const XY n0 = edge_node(G, cm.nx, cm.ny, 0, s);
    double b0, b1;
    body_at<FIELDS>(cm, n0.y * cm.nx + n0.x, n, a.r_n, b0, b1);
    R Uw[6];
    if constexpr (LINES) {
        // level n+1 of the two-level step, from the wall line of the staging buffer
        const T* lv = (const T*)wall_lines(a.aux, cm.nx, cm.ny).lines + line_slot(cm.nx, cm.ny, e, 0, s) * 24;
        recover_vals<T, R>(lv, 1, hdt * R(b0), hdt * R(b1), Uw);
    } else {
        recover_node<T, R>((const T*)a.pop, cm.ntile, n0.x, n0.y, hdt * R(b0), hdt * R(b1), Uw);
    }
    R tang[2], acol[2], Tv[2];
    for (int k = 0; k < 2; ++k) {
        tang[k] = Uw[2 + 2 * k + Bx];
        acol[k] = Uw[2 + 2 * k + AX];
        Tv[k] = edge_value<R>(a.ed, e, k, s, L);
    }
    R mu, lam;
    params_at<FIELDS, R>(cm, n0.y * cm.nx + n0.x, mu, lam);
    const bool ok = newton_column<R, LAW, SH, AX>(R(G.NA), tang, Tv, mu, lam, law_consts<R>(cm), acol,
                                                 cm.newton_max_iter, R(cm.newton_tol));
    if (!ok) atomicOr(cm.fault, (uint32_t)LBM_FAULT_NEWTON);
    R* aux = (R*)a.aux + 4 * (int64_t)(edge_off(cm.nx, cm.ny, e) + s);
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
// (the wall links and the collision of a node: lbm_collide.hpp)

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
        if (a.dUdX) {
            dX[k] = a.dUdX[k * n + idx];
            dY[k] = a.dUdY[k * n + idx];
        } else {
            dX[k] = fd_along<double>([&](int s) { return pl[int64_t(y) * nx + s]; }, x, nx, cm.periodic_x, inv2h);
            dY[k] = fd_along<double>([&](int s) { return pl[int64_t(s) * nx + x]; }, y, ny, cm.periodic_y, inv2h);
        }
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
        a.eblk[e + 1] = a.eblk[e] + (a.cm.bc[e] == LBM_TRACTION ? (L + kTracWin - 1) / kTracWin : 0);
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
    return launch_init_given(a, s);
}

// The populations from U0 already in a.scratch (and its derivatives, if given).
hipError_t launch_init_given(const InitArgs& a, hipStream_t s) {
    const dim3 grid(nblocks(int64_t(a.cm.nx) * a.cm.ny));
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: init_st<LBM_F32_SHIFTED>(a, s, grid); break;
        case LBM_F16_SHIFTED: init_st<LBM_F16_SHIFTED>(a, s, grid); break;
        default: init_st<LBM_F64_PLAIN>(a, s, grid); break;
    }
    return hipGetLastError();
}

}  // namespace lbm
