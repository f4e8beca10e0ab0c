// Device helpers shared by the forward and adjoint kernels: tile order, boundary data,
// per-node parameters, state recovery from stored populations, the traction-boundary
// Newton solve and the geometry of the half-way walls.
#pragma once

#include "lbm_device.hpp"
#include "lbm_internal.hpp"

namespace lbm {

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD b mod 8);
// hand XCD x the contiguous tile range [x per, (x + 1) per).
__device__ __forceinline__ int remap_tile(int b, int nb) {
    const int per = nb >> 3;
    if (b >= per * 8) return b;
    return (b & 7) * per + (b >> 3);
}

// v mod n in [0, n) for any v (periodic index).
__device__ __forceinline__ int wrap_index(int v, int n) {
    const int m = v % n;
    return m < 0 ? m + n : m;
}

// wrap_index for v >= -n, with the division only where v >= 2n (a lane index beyond a grid
// narrower than one tile): one compare and subtract in the common case.
__device__ __forceinline__ int wrap_near(int v, int n) {
    if (v < 0) return v + n;
    if (v < n) return v;
    v -= n;
    if (v < n) return v;
    return v % n;
}

// The neighbours x - 1 and x + 1 of 0 <= x < n on a periodic axis.
__device__ __forceinline__ int wrap_dec(int x, int n) { return x == 0 ? n - 1 : x - 1; }
__device__ __forceinline__ int wrap_inc(int x, int n) { return x + 1 == n ? 0 : x + 1; }

template <typename R>
__device__ __forceinline__ R edge_value(const EdgeData& ed, int e, int comp, int s, int L) {
    const double* f = ed.field[e];
    return f ? R(f[comp * L + s]) : R(ed.value[e][comp]);
}

// r b(X) of node idx: r times the body field, or the uniform value.
template <bool FIELDS>
__device__ __forceinline__ void body_at(const Common& cm, int idx, int64_t n, double r, double& b0, double& b1) {
    if (FIELDS && cm.body) {
        b0 = r * double(cm.body[idx]);
        b1 = r * double(cm.body[n + idx]);
    } else {
        b0 = r * cm.b0[0];
        b1 = r * cm.b0[1];
    }
}

// r b(X) of node idx in the compute type: r times the field (in double, then rounded), or
// the uniform r b0, which the host forms and rounds for R = float (fb).
template <bool FIELDS, typename R>
__device__ __forceinline__ void body_r(const Common& cm, int idx, int64_t n, double r, const float fb[2], R& B0,
                                       R& B1) {
    if (FIELDS && cm.body) {
        B0 = R(r * double(cm.body[idx]));
        B1 = R(r * double(cm.body[n + idx]));
    } else {
        B0 = kval<R>(r * cm.b0[0], fb[0]);
        B1 = kval<R>(r * cm.b0[1], fb[1]);
    }
}

template <bool FIELDS, typename R>
__device__ __forceinline__ void params_at(const Common& cm, int idx, R& mu, R& lam) {
    if (FIELDS && cm.mu) mu = R(cm.mu[idx]); else mu = kval<R>(cm.mu0, cm.f_mu0);
    if (FIELDS && cm.lam) lam = R(cm.lam[idx]); else lam = kval<R>(cm.lam0, cm.f_lam0);
}

template <typename R>
__device__ __forceinline__ LawK<R> law_consts(const Common& cm) {
    return LawK<R>{kval<R>(cm.law_k[0], cm.f_law_k[0]), kval<R>(cm.law_k[1], cm.f_law_k[1]),
                   kval<R>(cm.law_k[2], cm.f_law_k[2])};
}

// Sum of the four stored post-collision populations of one node minus (dt/2) B: the
// state of that level (sum_q f* = U + (dt/2) B, from eq:collision with sum_q w = 1/2).
template <typename T, typename R>
__device__ __forceinline__ void recover_vals(const T* p, int64_t stride, R hb0, R hb1, R U[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        R s = R(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) s += R(p[(6 * q + k) * stride]);
        U[k] = s;
    }
    U[0] -= hb0;
    U[1] -= hb1;
}

template <typename T, typename R>
__device__ __forceinline__ void recover_node(const T* pop, int ntile, int x, int y, R hb0, R hb1, R U[6]) {
    recover_vals<T, R>(pop + tile_base(ntile, 24, x, y), kTile, hb0, hb1, U);
}

// ---------------------------------------------------------------- traction Newton
// Normal column a = F^b_{.A} of the boundary deformation gradient from
// N_A P_iA(F^b) = T_i (Sec. 3.6, eq:neumann-boundary-rule).  Newton steps
// delta = -J^{-1} r with J_ik = N_A C_iAkA; step lengths 1, 1/2, ..., 2^-10, the first with
// det F^b > 0 and a smaller |r| is taken; stop at |r| <= tol (|T| + mu |F^b - I|), when no
// step length is accepted, or after max_iter updates.  Returns false on failure.  The axis
// A is a template parameter: indexed at run time, F and the tangent would live in scratch
// memory, one round trip per access inside the iteration.
template <typename R, int LAW, bool SH, int A>
__device__ bool newton_column(R NA, const R tang[2], const R T[2], R mu, R lam,
                              const LawK<R>& lk, R a[2], int max_iter, R tol) {
    constexpr int B = 1 - A;
    auto assemble = [&](const R ac[2], R f[4]) {
        f[A] = ac[0]; f[2 + A] = ac[1];
        f[B] = tang[0]; f[2 + B] = tang[1];
    };
    auto resid = [&](const R ac[2], R r[2], R& J) {
        R f[4], P[4];
        assemble(ac, f);
        piola<R, LAW, SH>(f, mu, lam, lk, P, J);
        r[0] = NA * P[A] - T[0];
        r[1] = NA * P[2 + A] - T[1];
    };
    auto scale = [&](const R ac[2]) {
        R f[4];
        assemble(ac, f);
        R s2;
        if constexpr (SH) s2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2] + f[3] * f[3];
        else s2 = (f[0] - R(1)) * (f[0] - R(1)) + f[1] * f[1] + f[2] * f[2] + (f[3] - R(1)) * (f[3] - R(1));
        return sqrt_r(T[0] * T[0] + T[1] * T[1]) + mu * sqrt_r(s2);
    };
    R r[2], J;
    resid(a, r, J);
    for (int it = 0; it < max_iter; ++it) {
        const R rn = sqrt_r(r[0] * r[0] + r[1] * r[1]);
        if (rn <= tol * scale(a)) break;
        R f[4], C[16];
        assemble(a, f);
        tangent<R, LAW, SH>(f, mu, lam, lk, C);
        const R j00 = NA * C[4 * A + A], j01 = NA * C[4 * A + 2 + A];
        const R j10 = NA * C[8 + 4 * A + A], j11 = NA * C[8 + 4 * A + 2 + A];
        const R det = j00 * j11 - j01 * j10;
        const R d0 = -(j11 * r[0] - j01 * r[1]) / det;
        const R d1 = -(-j10 * r[0] + j00 * r[1]) / det;
        R alpha = R(1);
        bool accepted = false;
        for (int ls = 0; ls < 11; ++ls) {
            const R trial[2] = {a[0] + alpha * d0, a[1] + alpha * d1};
            R rt[2], Jt;
            resid(trial, rt, Jt);
            if (Jt > R(0) && sqrt_r(rt[0] * rt[0] + rt[1] * rt[1]) < rn) {
                a[0] = trial[0]; a[1] = trial[1];
                r[0] = rt[0]; r[1] = rt[1];
                J = Jt;
                accepted = true;
                break;
            }
            alpha *= R(0.5);
        }
        if (!accepted) break;
    }
    const R rn = sqrt_r(r[0] * r[0] + r[1] * r[1]);
    // With the plain F the residual cannot drop below the rounding of terms of size
    // |T| + 2 mu (P subtracts O(mu) quantities); the shifted form has no such floor.
    const R eps = sizeof(R) == 8 ? R(2.220446049250313e-16) : R(1.1920929e-7);
    const R floor = SH ? R(0) : R(1e3) * eps * (sqrt_r(T[0] * T[0] + T[1] * T[1]) + R(2) * mu);
    return (rn <= R(1e-4) * scale(a) + floor) && (J > R(0)) && finite_r(rn);
}

// Node (x, y) of row r (0 = wall row, 1 = first interior row) at position s2 of edge e.
struct XY {
    int x, y;
};
__device__ __forceinline__ XY edge_node(const EdgeGeom& G, int nx, int ny, int r, int s2) {
    if (G.A == 0) return XY{(G.NA < 0) ? r : nx - 1 - r, s2};
    return XY{s2, (G.NA < 0) ? r : ny - 1 - r};
}

// Wall lines of the two-level step on grids with walls.  The staging buffer (aux) holds,
// after the F^b of every link (4 values of 8 bytes each), the populations of level n+1 on
// the wall line (r = 0) and the first interior line (r = 1) of every edge, 24 values of
// 8 bytes per node, and the state U^{n+1} of the wall-line nodes, 6 values of 8 bytes:
//   line value p of node s of line r of edge e at  lines + (2 off[e] + r len[e] + s) 24 + p
//   U^{n+1} component k of wall node s of edge e at u1 + (off[e] + s) 6 + k
// (off, len from edge_offsets, in links).
struct WallLines {
    char* lines;
    char* u1;
};

__host__ __device__ inline WallLines wall_lines(void* aux, int nx, int ny) {
    const int64_t links = 2 * int64_t(nx) + 2 * int64_t(ny);
    WallLines w;
    w.lines = (char*)aux + links * 4 * 8;
    w.u1 = w.lines + links * 2 * 24 * 8;
    return w;
}

__host__ __device__ inline int64_t line_slot(int nx, int ny, int e, int r, int s) {
    return 2 * int64_t(edge_off(nx, ny, e)) + int64_t(r) * edge_len(nx, ny, e) + s;
}

// A line of a wall edge that holds node (x, y): the first of XMIN, XMAX, YMIN, YMAX whose
// wall line or first interior line passes through it.
__device__ __forceinline__ bool find_line(const Common& cm, int x, int y, int& e, int& r, int& s) {
    if (!cm.periodic_x) {
        if (x <= 1) { e = LBM_XMIN; r = x; s = y; return true; }
        if (x >= cm.nx - 2) { e = LBM_XMAX; r = cm.nx - 1 - x; s = y; return true; }
    }
    if (!cm.periodic_y) {
        if (y <= 1) { e = LBM_YMIN; r = y; s = x; return true; }
        if (y >= cm.ny - 2) { e = LBM_YMAX; r = cm.ny - 1 - y; s = x; return true; }
    }
    return false;
}

// Tile-grid position of this thread for kernels with one wavefront per tile and
// blockDim.x / 64 tiles per workgroup.  Returns false for lanes beyond the grid.
__device__ __forceinline__ bool tile_thread(int nx, int ny, int ntile, int& x, int& y) {
    const int tl = remap_tile(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tl >= ntile * ny) return false;
    y = tl / ntile;
    x = (tl - y * ntile) * kTile + (threadIdx.x & (kTile - 1));
    return x < nx;
}

}  // namespace lbm
