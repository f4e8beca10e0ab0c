// Several levels of the fused collide-stream per pass over HBM on periodic grids
// (lbm_step_multi).  A wavefront owns a window of 64 columns and a segment of rows and
// marches down the segment: each iteration pulls one new row of f*^n from memory, takes it
// to level n+1, and takes the rows behind it one level further each, so that the levels in
// between never leave registers.  Every node's arithmetic is collide_node, as in
// step_kernel, and each intermediate level is rounded to the storage type, so the result is
// bit for bit that of as many single steps.
#include "lbm_collide.hpp"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"
#include "lbm_march.hpp"

namespace lbm {

// The LDS of one workgroup: the output row of its span, in the storage type, and the
// accumulator words of that row; two buffers (one for FP64, whose row is twice as large)
// so that one barrier per iteration separates the writes of a row from its reads.
template <int ST, int NT, bool REC>
struct MarchLds {
    static constexpr int nbuf = ST == LBM_F64_PLAIN ? 1 : 2;
    __attribute__((aligned(16))) typename Storage<ST>::pop_t pop[nbuf][24][kMarchSpan];
    __attribute__((aligned(16))) float S[nbuf][2][kMarchSpan];
    __attribute__((aligned(16))) double U[nbuf][2][kMarchSpan];
};
// The replay form (REC: records of every level, no displacement accumulator): the output
// row of the populations and the rows of the records of the NT levels.  Where two buffers
// of records do not fit the 160 KB of LDS beside the two population rows (four FP32 levels:
// 86 KB of records, 86 KB of populations), they have one, and a second barrier per
// iteration follows their stores.
template <int ST, int NT>
struct MarchLds<ST, NT, true> {
    static constexpr int nbuf = 2;
    static constexpr int rbuf =
        2 * 24 * kMarchSpan * sizeof(typename Storage<ST>::pop_t) + 2 * NT * 6 * kMarchSpan * sizeof(float) <=
                160 * 1024 ? 2 : 1;
    __attribute__((aligned(16))) typename Storage<ST>::pop_t pop[2][24][kMarchSpan];
    __attribute__((aligned(16))) float rec[rbuf][NT][6][kMarchSpan];
};

template <int ST, int NT, bool REC> constexpr int rec_buffers() {
    if constexpr (REC) return MarchLds<ST, NT, true>::rbuf;
    else return 0;
}

// Geometry.  A workgroup owns a span of kMarchTiles = 7 aligned tiles (448 columns) and a
// segment of rows; its kMarchWaves = 8 wavefronts each compute a window of 64 columns.
// Level n+1 is pulled from memory on all 64 lanes; a later level pulls its x-neighbours
// from the adjacent lanes, so each level loses one lane at either end and level n+NT is
// complete on lanes [NT-1, 64-NT]: a window outputs OW = 64 - 2 (NT - 1) columns.  Windows
// 0 .. 6 output the columns [k OW, (k + 1) OW) of the span and window 7 its last OW
// columns, which covers the span for NT <= 5.  The output rows go through LDS, and
// wavefront k < 7 stores tile k of the span whole: stores of parts of a tile from two
// wavefronts cost several times the bytes they move.
//
// Rows.  Iteration i takes row y1 = Y0 - (NT - 1) + i to level n+1 and row y1 - (L - 1) to
// level n+L.  Level n+L of row y needs level n+L-1 of rows y - 1, y and y + 1: row y + 1 was
// taken to that level earlier in the same iteration, row y one iteration and row y - 1 two
// iterations before (kept in registers: the planes q1 of two rows, q0 and q2 of one row,
// already shifted across lanes).  Level n+L runs from iteration 2 (L - 1) on, and the
// segment's S output rows take S + 2 (NT - 1) iterations.
//
// Memory operations.  The loads of an iteration's new row are issued one iteration ahead,
// before the previous iteration's stores.  Loads and stores share one wait counter, which
// counts in issue order, so the wait for those loads need not wait for the stores as long
// as every path through the loop issues the same stores after them: the compiler sizes the
// wait for the path with the fewest.  Hence every iteration stores a full tile row on every
// lane of every wavefront (lanes, wavefronts and iterations without output store to
// kNoStore), and before the loop one such row of empty stores follows the first loads.
//
// REC (the replay of the checkpointed adjoint): no displacement accumulator; the record of
// every level (v and F - I, as lbm_step writes it) goes through LDS like the output row
// and is stored whole per tile for the rows of the segment.
template <int ST, int LAW, bool FIELDS, int NT, bool REC>
__global__ void __launch_bounds__(kMarchWaves * kTile) march_kernel(MarchArgs a) {
    using Tr = Storage<ST>;
    using R = typename Tr::real;
    using T = typename Tr::pop_t;
    constexpr bool SH = Tr::shifted;
    constexpr int OW = kTile - 2 * (NT - 1);
    static_assert(kMarchTiles * OW + OW >= kMarchSpan, "the windows must cover the span");
    constexpr uint32_t kPlane = kTile * sizeof(T);     // bytes between planes of a tile
    static_assert(!REC || SH, "records of the shifted storages only");
    constexpr int NB = MarchLds<ST, NT, REC>::nbuf;
    constexpr int NRB = rec_buffers<ST, NT, REC>();
    auto record_buffer = [](int i) { return NRB == 1 ? 0 : (i & 1); };
    __shared__ MarchLds<ST, NT, REC> sh;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny, ntile = cm.ntile;
    const int64_t n = int64_t(nx) * ny;
    const int lane = threadIdx.x & (kTile - 1);
    // the wavefront index, known to the compiler to be uniform: the rows, the segment and the
    // loop count then live in scalar registers
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = remap_tile(blockIdx.x, gridDim.x);
    if (g >= a.nwg) return;
    const int seg = fdiv(g, a.d_nspan), span = g - seg * a.nspan;
    const int c0 = span * kMarchSpan;                   // first column of the span
    const int ws = w < kMarchTiles ? w * OW : kMarchSpan - OW;   // window's first output column
    const int xg = c0 + ws - (NT - 1) + lane;
    const int xc = wrap_index(xg, nx);
    const int om = pop_col(wrap_dec(xc, nx)), oc = pop_col(xc), op = pop_col(wrap_inc(xc, nx));
    const int64_t rowe = int64_t(ntile) * 24 * kTile;  // elements per row of population tiles
    const int64_t rowu = int64_t(ntile) * 2 * kTile;   // elements per row of the u* planes
    const int ou = (xc >> 6) * (2 * kTile) + (xc & (kTile - 1));
    const int Y0 = seg * a.seg, Sy = min(a.seg, ny - Y0);
    // this lane's output column in the span (window 7 leaves the columns of window 6 to it)
    const int pos = ws - (NT - 1) + lane;
    const bool out_lane = lane >= NT - 1 && lane <= kTile - NT &&
                          (w < kMarchTiles || pos >= (kMarchTiles - 1) * OW + OW);
    // the tile this wavefront stores (wavefront 7 stores none)
    const int st = c0 / kTile + w;
    const T* __restrict__ src = (const T*)a.src;
    T* __restrict__ dst = (T*)a.dst;
    float* Sbase = (float*)a.ustar;                     // shifted storages: S, then U
    double* Ubase = ST == LBM_F64_PLAIN ? (double*)a.ustar
                                        : (double*)(Sbase + 2 * int64_t(ntile) * kTile * ny);
    const R dt = kval<R>(cm.dt, cm.f_dt);
    const bool any_fold = ST != LBM_F64_PLAIN && (a.fold[0] | a.fold[1] | a.fold[2] | a.fold[3]);

    // rw[j]: row y1 + 1 - j, wrapped (wave-uniform)
    int rw[NT + 1];
#pragma unroll
    for (int j = 0; j <= NT; ++j) rw[j] = wrap_index(Y0 - (NT - 1) + 1 - j, ny);

    // The pulled populations of level n for the next row to enter level n+1 (q0 from x-1,
    // q2 from x+1 of row y1, q1 from row y1 - 1, q3 from row y1 + 1; eq:streaming), with
    // its per-node parameters, and the accumulator words of the next output row.
    T pre[24];
    float pprm[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float pS[2] = {0.0f, 0.0f};
    double pU[2] = {0.0, 0.0};
    auto prefetch = [&](int yp, int yc, int ym, int yo) {
        const T* rc = src + yc * rowe;
        const T* rm = src + ym * rowe;
        const T* rp = src + yp * rowe;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            pre[k] = rc[om + k * kTile];
            pre[12 + k] = rc[op + (12 + k) * kTile];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            pre[6 + k] = rm[oc + (6 + k) * kTile];
            pre[18 + k] = rp[oc + (18 + k) * kTile];
        }
        if constexpr (FIELDS) {
            const int idx = yc * nx + xc;
            if (cm.mu) pprm[0] = cm.mu[idx];
            if (cm.lam) pprm[1] = cm.lam[idx];
            if (cm.body) {
                pprm[2] = cm.body[idx];
                pprm[3] = cm.body[n + idx];
            }
        }
        if constexpr (REC) {
        } else if constexpr (ST == LBM_F64_PLAIN) {
            const double* us = Ubase + yo * rowu + ou;
            pU[0] = us[0];
            pU[1] = us[kTile];
        } else {
            const float* S = Sbase + yo * rowu + ou;
            pS[0] = S[0];
            pS[1] = S[kTile];
            if (any_fold) {
                const double* U = Ubase + yo * rowu + ou;
                pU[0] = U[0];
                pU[1] = U[kTile];
            }
        }
    };
    // The stores of output row yo from LDS buffer b: tile st of the populations and of the
    // accumulator words (byte offsets kNoStore where nothing is stored), in 16-byte pieces,
    // 1 KB per instruction (the 24 planes of a tile are contiguous).  The tile is stored
    // whole, so that a tile the grid's last column cuts receives values in its padding
    // columns (wrapped copies of real nodes, never read).  No branch may choose between
    // store sequences of different lengths here: the compiler's waits would then assume the
    // shortest, and a path that skips both would be taken as possible.
    auto store_row = [&](int yo, bool outp, int b, bool moved, int outp_iter) {
        const bool on = outp && w < kMarchTiles && st < ntile;
        const __amdgpu_buffer_rsrc_t rp = row_rsrc(dst + yo * rowe, rowe * int64_t(sizeof(T)));
        const uint32_t tb = uint32_t(st * 24 * kTile) * uint32_t(sizeof(T));   // tile's first byte
        const int lc = w < kMarchTiles ? w * kTile : 0;                      // tile's LDS column
        constexpr int V = 16 / sizeof(T);          // elements per 16-byte piece
        constexpr int LPP = kTile / V;             // lanes per plane
        constexpr int PPI = kTile / LPP;           // planes per instruction
#pragma unroll
        for (int j = 0; j < 24 / PPI; ++j) {
            const int p = j * PPI + lane / LPP, col = (lane % LPP) * V;
            const u32x4 v = *(const u32x4*)&sh.pop[b][p][lc + col];
            row_store16(rp, on ? tb + uint32_t(p * kTile + col) * uint32_t(sizeof(T)) : kNoStore, v);
        }
        if constexpr (REC) {
            // the record rows of the levels whose rows lie in the segment: 6 planes of 64
            // words per tile, planes 0 .. 3 in one instruction and 4, 5 on half the lanes
            // (with rec_planes = 4 the velocity planes 0, 1 are left out)
            const int pl = lane >> 4, col = (lane & 15) * 4;
            const int64_t rowr = int64_t(ntile) * 6 * kTile;
            const int rb = NRB == 1 ? 0 : b;
#pragma unroll
            for (int L = 1; L <= NT; ++L) {
                const int i0 = NT + L - 2;                  // first iteration of a segment row
                const bool rin = outp_iter >= i0 && outp_iter < i0 + Sy && w < kMarchTiles && st < ntile;
                const __amdgpu_buffer_rsrc_t rr = row_rsrc((float*)a.rec[L - 1] + rw[L] * rowr, rowr * 4);
                const uint32_t tr = uint32_t(st * 6 * kTile);
                const u32x4 v0 = *(const u32x4*)&sh.rec[rb][L - 1][pl][lc + col];
                row_store16(rr, rin && (pl >= 2 || a.rec_planes == 6) ? (tr + uint32_t(pl * kTile + col)) * 4u
                                                                     : kNoStore, v0);
                const int p1 = 4 + (pl & 1);
                const u32x4 v1 = *(const u32x4*)&sh.rec[rb][L - 1][p1][lc + col];
                row_store16(rr, rin && pl < 2 ? (tr + uint32_t(p1 * kTile + col)) * 4u : kNoStore, v1);
            }
        } else {
            // two u* planes of 64 words: 32 lanes per plane
            const int cp = lane >> 5, cc = (lane & 31) * 2;
            const uint32_t uw = uint32_t(st * 2 * kTile + cp * kTile + cc);
            if constexpr (ST != LBM_F64_PLAIN) {
                const __amdgpu_buffer_rsrc_t rs = row_rsrc(Sbase + yo * rowu, rowu * 4);
                const u32x2 v = *(const u32x2*)&sh.S[b][cp][lc + cc];
                row_store8(rs, on ? uw * 4u : kNoStore, v);
            }
            if (ST == LBM_F64_PLAIN || moved) {
                const __amdgpu_buffer_rsrc_t ru = row_rsrc(Ubase + yo * rowu, rowu * 8);
                const u32x4 v = *(const u32x4*)&sh.U[b][cp][lc + cc];
                row_store16(ru, on ? uw * 8u : kNoStore, v);
            }
        }
    };
    // parameters (mu, lam, body) of the rows of levels n+1 .. n+NT, newest first
    float prm[NT][4];
#pragma unroll
    for (int L = 0; L < NT; ++L) prm[L][0] = prm[L][1] = prm[L][2] = prm[L][3] = 0.0f;
    auto node_params = [&](int L, R& B0, R& B1, R& mu, R& lam) {
        if (FIELDS && cm.body) {
            B0 = R(a.r[L] * double(prm[L][2]));
            B1 = R(a.r[L] * double(prm[L][3]));
        } else {
            B0 = kval<R>(a.r[L] * cm.b0[0], a.fb[L][0]);
            B1 = kval<R>(a.r[L] * cm.b0[1], a.fb[L][1]);
        }
        if (FIELDS && cm.mu) mu = R(prm[L][0]); else mu = kval<R>(cm.mu0, cm.f_mu0);
        if (FIELDS && cm.lam) lam = R(prm[L][1]); else lam = kval<R>(cm.lam0, cm.f_lam0);
    };

    // level n+L (L = 1 .. NT-1) of the rows behind: q1 of the last two rows, q0 and q2 of the
    // last row shifted to the lanes that pull them
    R hq1a[NT - 1][6], hq1b[NT - 1][6], ho0[NT - 1][6], ho2[NT - 1][6];
    // velocity of level n+L (L < NT) of the last NT - L rows, newest first
    R vh[NT][NT][2];
#pragma unroll
    for (int L = 0; L < NT - 1; ++L)
#pragma unroll
        for (int k = 0; k < 6; ++k) hq1a[L][k] = hq1b[L][k] = ho0[L][k] = ho2[L][k] = R(0);
#pragma unroll
    for (int L = 0; L < NT; ++L)
#pragma unroll
        for (int j = 0; j < NT; ++j) vh[L][j][0] = vh[L][j][1] = R(0);
    bool nonfinite = false, jbad = false;

    const int iters = Sy + 2 * (NT - 1);
    // A window that starts past the last stored tile (in a row's last span) outputs no
    // column of a stored tile, and its own tile is not stored either (a window starts no
    // later than its tile): the wavefront only takes part in the workgroup's barriers.  A
    // window that starts past the grid's last column but inside the last tile still runs,
    // so that the padding columns of that tile receive the wrapped copies of real nodes
    // and every stored word is defined.
    if (c0 + ws >= ntile * kTile) {
        for (int i = 0; i < iters; ++i) {
            if (NB == 1) __syncthreads();
            __syncthreads();
            if constexpr (REC && NRB == 1) __syncthreads();
        }
        return;
    }
    prefetch(rw[0], rw[1], rw[2], rw[NT]);
    store_row(rw[NT], false, 0, false, -1);
    auto iteration = [&](int i, auto steady_c) {
        constexpr bool steady = decltype(steady_c)::value;
        const int b = NB == 1 ? 0 : (i & 1);
        const int rb = record_buffer(i);
        // REC: the record of level t at this lane's output column into LDS buffer b
        auto stage_record = [&](int t, const R Uv[6]) {
            if constexpr (REC) {
                if (out_lane) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) sh.rec[rb][t][k][pos] = Uv[k];
                }
            }
        };
        R f[4][6], U[6], J;
        R cv[NT][2] = {};
        R gq[4][6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            gq[0][k] = R(pre[k]);
            gq[1][k] = R(pre[6 + k]);
            gq[2][k] = R(pre[12 + k]);
            gq[3][k] = R(pre[18 + k]);
        }
        if constexpr (FIELDS) {
#pragma unroll
            for (int L = NT - 1; L >= 1; --L)
#pragma unroll
                for (int c = 0; c < 4; ++c) prm[L][c] = prm[L - 1][c];
#pragma unroll
            for (int c = 0; c < 4; ++c) prm[0][c] = pprm[c];
        }
        const float Sp[2] = {pS[0], pS[1]};
        const double Up[2] = {pU[0], pU[1]};
        // the next iteration's rows y1 + 2, y1 + 1 and y1 and its output row (on the last
        // iteration a row that is not used: every iteration issues the same loads)
        prefetch(wrap_inc(rw[0], ny), rw[0], rw[1], rw[NT - 1]);
        {
            // level n+1 of row y1
            R B0, B1, mu, lam;
            node_params(0, B0, B1, mu, lam);
            collide_node<R, LAW, SH>(cm, gq, B0, B1, mu, lam, f, U, J);
#pragma unroll
            for (int k = 0; k < 6; ++k) nonfinite |= !finite_r(U[k]);
            jbad |= J <= R(0);
            cv[0][0] = U[0];
            cv[0][1] = U[1];
            stage_record(0, U);
        }
#pragma unroll
        for (int L = 2; L <= NT; ++L) {
            if (!steady && i < 2 * (L - 2)) break;  // level n+L-1 has not started
            // f: level n+L-1 of row y1 - (L - 2), rounded to the stored value
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < 6; ++k) f[q][k] = R(to_storage<T>(f[q][k]));
            const bool act = steady || i >= 2 * (L - 1);
            if (act) {
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    gq[0][k] = ho0[L - 2][k];
                    gq[1][k] = hq1b[L - 2][k];
                    gq[2][k] = ho2[L - 2][k];
                    gq[3][k] = f[3][k];
                }
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                hq1b[L - 2][k] = hq1a[L - 2][k];
                hq1a[L - 2][k] = f[1][k];
                ho0[L - 2][k] = from_prev(f[0][k]);
                ho2[L - 2][k] = from_next(f[2][k]);
            }
            if (!act) break;
            R B0, B1, mu, lam;
            node_params(L - 1, B0, B1, mu, lam);
            collide_node<R, LAW, SH>(cm, gq, B0, B1, mu, lam, f, U, J);
            // level n+L is complete on lanes [L - 1, 64 - L]
            if (lane >= L - 1 && lane <= kTile - L) {
#pragma unroll
                for (int k = 0; k < 6; ++k) nonfinite |= !finite_r(U[k]);
                jbad |= J <= R(0);
            }
            cv[L - 1][0] = U[0];
            cv[L - 1][1] = U[1];
            stage_record(L - 1, U);
        }
        // f: level n+NT of output row y1 - (NT - 1) from iteration 2 (NT - 1) on.  The
        // displacement quadrature over the NT levels (eq:trapezoid-u), with the accumulator
        // updates and folds of NT single steps.
        const bool outp = steady || i >= 2 * (NT - 1);
        float Sn[2] = {0.0f, 0.0f};
        double Un[2] = {0.0, 0.0};
        bool moved = false;
#pragma unroll
        for (int cpt = 0; cpt < 2; ++cpt) {
            if constexpr (REC) {
            } else if constexpr (ST == LBM_F64_PLAIN) {
                double s = Up[cpt];
#pragma unroll
                for (int L = 1; L <= NT; ++L) s = s + dt * (L == NT ? cv[NT - 1][cpt] : vh[L - 1][NT - L - 1][cpt]);
                Un[cpt] = s;
            } else {
                float sn = Sp[cpt];
                double u = 0.0;
                bool mv = false;
#pragma unroll
                for (int L = 1; L <= NT; ++L) {
                    const R v = L == NT ? cv[NT - 1][cpt] : vh[L - 1][NT - L - 1][cpt];
                    sn = sn + float(dt * v);
                    if (a.fold[L - 1]) {
                        u = (mv ? u : Up[cpt]) + double(sn);
                        sn = 0.0f;
                        mv = true;
                    }
                }
                Sn[cpt] = sn;
                Un[cpt] = u;
                moved = mv;
            }
        }
        if (NB == 1) __syncthreads();               // the previous row has been read
        if (outp && out_lane) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < 6; ++k) sh.pop[b][6 * q + k][pos] = to_storage<T>(f[q][k]);
            if constexpr (!REC) {
                if constexpr (ST != LBM_F64_PLAIN) {
                    sh.S[b][0][pos] = Sn[0];
                    sh.S[b][1][pos] = Sn[1];
                }
                sh.U[b][0][pos] = Un[0];
                sh.U[b][1][pos] = Un[1];
            }
            if (lane >= NT - 1 && lane <= kTile - NT) {
#pragma unroll
                for (int k = 0; k < 6; ++k) nonfinite |= !finite_r(U[k]);
                jbad |= J <= R(0);
            }
        }
        __syncthreads();
        store_row(rw[NT], outp, b, moved, i);
        // one buffer of records: every wavefront has read them before the next are staged
        if constexpr (REC && NRB == 1) __syncthreads();
        // the velocity history moves one row on
#pragma unroll
        for (int L = 1; L < NT; ++L) {
#pragma unroll
            for (int j = NT - L - 1; j >= 1; --j) {
                vh[L - 1][j][0] = vh[L - 1][j - 1][0];
                vh[L - 1][j][1] = vh[L - 1][j - 1][1];
            }
            vh[L - 1][0][0] = cv[L - 1][0];
            vh[L - 1][0][1] = cv[L - 1][1];
        }
#pragma unroll
        for (int j = NT; j >= 1; --j) rw[j] = rw[j - 1];
        rw[0] = wrap_inc(rw[0], ny);
    };
    // (the invariant-based laws, short of registers already, keep one loop: a second copy
    // of the body made them spill more)
    constexpr bool kPeel = LAW == LBM_LOGNH || LAW == LBM_NH || LAW == LBM_SVK;
    int i = 0;
    if constexpr (kPeel) {
        const int warm = iters < 2 * (NT - 1) ? iters : 2 * (NT - 1);
        for (; i < warm; ++i) iteration(i, std::false_type{});
        for (; i < iters; ++i) iteration(i, std::true_type{});
    } else {
        for (; i < iters; ++i) iteration(i, std::false_type{});
    }
    if (nonfinite || jbad)
        atomicOr(cm.fault, (jbad ? (uint32_t)LBM_FAULT_J : 0u) | (nonfinite ? (uint32_t)LBM_FAULT_NONFINITE : 0u));
}

// ---------------------------------------------------------------- dispatch

template <int ST, int LAW, bool FIELDS>
static hipError_t march_levels(const MarchArgs& a, hipStream_t s) {
    const dim3 grid(unsigned(a.nwg)), block(kMarchWaves * kTile);
    if (a.rec[0]) {
        // the replay form: records of every level, no accumulator
        if constexpr (ST != LBM_F64_PLAIN) {
            if (a.levels == 2) hipLaunchKernelGGL((march_kernel<ST, LAW, FIELDS, 2, true>), grid, block, 0, s, a);
            else if (a.levels == 3) hipLaunchKernelGGL((march_kernel<ST, LAW, FIELDS, 3, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((march_kernel<ST, LAW, FIELDS, 4, true>), grid, block, 0, s, a);
        }
        return hipGetLastError();
    }
    switch (a.levels) {
        case 2: hipLaunchKernelGGL((march_kernel<ST, LAW, FIELDS, 2, false>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((march_kernel<ST, LAW, FIELDS, 3, false>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((march_kernel<ST, LAW, FIELDS, 4, false>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

template <int ST, int LAW>
static hipError_t march_st_law(const MarchArgs& a, hipStream_t s) {
    const bool fields = a.cm.mu || a.cm.lam || a.cm.body;
    return fields ? march_levels<ST, LAW, true>(a, s) : march_levels<ST, LAW, false>(a, s);
}

template <int ST>
static hipError_t march_st(const MarchArgs& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: return march_st_law<ST, LBM_LOGNH>(a, s);
        case LBM_NH: return march_st_law<ST, LBM_NH>(a, s);
        case LBM_MR: return march_st_law<ST, LBM_MR>(a, s);
        case LBM_YEOH: return march_st_law<ST, LBM_YEOH>(a, s);
        case LBM_GENT: return march_st_law<ST, LBM_GENT>(a, s);
        default: return march_st_law<ST, LBM_SVK>(a, s);
    }
}

hipError_t launch_march(const MarchArgs& a, hipStream_t s) {
    switch (a.cm.storage) {
        case LBM_F32_SHIFTED: return march_st<LBM_F32_SHIFTED>(a, s);
        case LBM_F16_SHIFTED: return march_st<LBM_F16_SHIFTED>(a, s);
        default: return march_st<LBM_F64_PLAIN>(a, s);
    }
}

}  // namespace lbm
