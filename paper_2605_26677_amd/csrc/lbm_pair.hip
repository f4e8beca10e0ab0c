// Two levels of the fused collide-stream per pass over HBM (lbm_step2): the workgroup
// kernels for periodic grids and for the interior and rim of walled grids, the wall-node
// pass, and their dispatch.  Every node's arithmetic is that of the single step
// (lbm_collide.hpp).
#include "lbm_collide.hpp"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"

namespace lbm {

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

// ---------------------------------------------------------------- dispatch

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

}  // namespace lbm
