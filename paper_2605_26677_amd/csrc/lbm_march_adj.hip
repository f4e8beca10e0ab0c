// Several levels of the hand-written adjoint per pass over HBM on periodic grids
// (lbm_adjoint_step_multi): the transpose of march_kernel.  A wavefront marches a window of
// 64 columns down a segment of rows; each iteration pulls one new row of lambda^{m+1} from
// memory and takes it to lambda^m, and takes the rows behind it one adjoint level further
// each, so that the levels in between never leave registers.  Every node's arithmetic is
// adj_node, as in adjoint_kernel, with the probe source and the gradient updates of each
// level in the order of single steps, so the result is bit for bit that of as many
// lbm_adjoint_step calls.
#include "lbm_adjoint.hpp"
#include "lbm_device.hpp"
#include "lbm_internal.hpp"
#include "lbm_kernel_util.hpp"
#include "lbm_march.hpp"

namespace lbm {

// The LDS of one workgroup: the output row of lambda and of the FP32 gradient block sums,
// two buffers so that one barrier per iteration separates the writes of a row from its
// reads; and, per lane, the running block sums of the rows between their first and last
// level (a ring of NT rows, each lane reading back only what it wrote).
template <int NT> struct MarchAdjLds {
    __attribute__((aligned(16))) float lam[2][24][kMarchSpan];
    __attribute__((aligned(16))) float gs[2][4][kMarchSpan];
    __attribute__((aligned(16))) float4 ring[NT][kMarchWaves][kTile];
};

// Geometry and memory operations as in march_kernel.  The adjoint pulls from X + c_q: level
// t+1 of row y takes q0 from x+1 and q2 from x-1 of row y (lanes shifted), q1 from row y+1
// (this iteration) and q3 from row y-1 (two iterations before).  Level t of the pass is
// adjoint level m - t and reads the record of U^{m-t}.  The FP32 compute type is the
// storage of lambda, so no level is rounded.
//
// Gradients (GRAD): a row's block sums are loaded with its first level and carried from
// level to level in the LDS ring; each level adds its increment, folds into the FP64
// gradients if it folds and then adds its probe body term, in the order of single steps;
// the last level stores the sums with lambda.
template <int ST, int LAW, bool FIELDS, int NT, bool GRAD>
__global__ void __launch_bounds__(kMarchWaves * kTile) march_adj_kernel(MarchAdjArgs a) {
    using R = float;
    constexpr int OW = kTile - 2 * (NT - 1);
    static_assert(ST != LBM_F64_PLAIN, "the FP32 compute type only");
    static_assert(kMarchTiles * OW + OW >= kMarchSpan, "the windows must cover the span");
    __shared__ MarchAdjLds<NT> sh;
    const Common& cm = a.cm;
    const int nx = cm.nx, ny = cm.ny, ntile = cm.ntile;
    const int64_t n = int64_t(nx) * ny;
    const int lane = threadIdx.x & (kTile - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = remap_tile(blockIdx.x, gridDim.x);
    if (g >= a.nwg) return;
    const int seg = fdiv(g, a.d_nspan), span = g - seg * a.nspan;
    const int c0 = span * kMarchSpan;
    const int ws = w < kMarchTiles ? w * OW : kMarchSpan - OW;
    const int xg = c0 + ws - (NT - 1) + lane;
    const int xc = wrap_index(xg, nx);
    const int om = pop_col(wrap_dec(xc, nx)), oc = pop_col(xc), op = pop_col(wrap_inc(xc, nx));
    const int orc = (xc >> 6) * (6 * kTile) + (xc & (kTile - 1));     // in a row of record tiles
    const int64_t rowe = int64_t(ntile) * 24 * kTile;
    const int64_t rowr = int64_t(ntile) * 6 * kTile;
    const int64_t rowg = int64_t(ntile) * 4 * kTile;
    const int og = (xc >> 6) * (4 * kTile) + (xc & (kTile - 1));      // in a row of block-sum tiles
    const int Y0 = seg * a.seg, Sy = min(a.seg, ny - Y0);
    const int pos = ws - (NT - 1) + lane;
    const bool out_lane = lane >= NT - 1 && lane <= kTile - NT &&
                          (w < kMarchTiles || pos >= (kMarchTiles - 1) * OW + OW);
    const int st = c0 / kTile + w;
    const R* __restrict__ src = (const R*)a.src;
    R* __restrict__ dst = (R*)a.dst;
    float* gsum = (float*)a.gsum;
    const bool gpar = a.g_mu || a.g_lam, gbody = a.g_body != nullptr;
    const bool has[4] = {a.g_mu != nullptr, a.g_lam != nullptr, gbody, gbody};
    double* const g64[4] = {a.g_mu, a.g_lam, a.g_body, a.g_body ? a.g_body + n : nullptr};
    const double hdt = 0.5 * cm.dt;

    int rw[NT + 1];
#pragma unroll
    for (int j = 0; j <= NT; ++j) rw[j] = wrap_index(Y0 - (NT - 1) + 1 - j, ny);

    // Loaded one iteration ahead, each right after the level that consumed the values before
    // (so that the two share registers): lambda^{m+1} pulled for the next row to enter level
    // m, mu and lam of that row and its block sums after level 0; the record and the
    // probe-table word of level t's next row after level t.
    float pre[24];
    float prec[NT][4];
    uint32_t pmw[NT];
    float pprm[2] = {0.0f, 0.0f};
    float pgs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    auto prefetch_row = [&](int yp, int yc, int ym) {
        const R* rc = src + yc * rowe;
        const R* rp = src + yp * rowe;
        const R* rm = src + ym * rowe;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            pre[k] = rc[op + k * kTile];
            pre[12 + k] = rc[om + (12 + k) * kTile];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            pre[6 + k] = rp[oc + (6 + k) * kTile];
            pre[18 + k] = rm[oc + (18 + k) * kTile];
        }
        if constexpr (FIELDS) {
            const int idx = yc * nx + xc;
            if (cm.mu) pprm[0] = cm.mu[idx];
            if (cm.lam) pprm[1] = cm.lam[idx];
        }
        if constexpr (GRAD) {
            const float* gp = gsum + yc * rowg + og;
#pragma unroll
            for (int j = 0; j < 4; ++j) pgs[j] = gp[j * kTile];
        }
    };
    auto prefetch_level = [&](int t, int yt) {
        const R* rec = (const R*)a.rec[t] + yt * rowr + orc;
#pragma unroll
        for (int k = 0; k < 4; ++k) prec[t][k] = rec[(2 + k) * kTile];
        // the 32-bit half of the probe-table word that holds bit x mod 64
        pmw[t] = a.pmask ? ((const uint32_t*)a.pmask)[2 * (int64_t(yt) * ntile + (xc >> 6)) + ((xc >> 5) & 1)] : 0u;
    };
    // the stores of output row yo from LDS buffer b (byte offsets kNoStore where nothing is
    // stored; see march_kernel): tile st of lambda and of the block sums, whole, in 16-byte
    // pieces
    auto store_row = [&](int yo, bool outp, int b) {
        const bool on = outp && w < kMarchTiles && st < ntile;
        const int lc = w < kMarchTiles ? w * kTile : 0;
        const __amdgpu_buffer_rsrc_t rl = row_rsrc(dst + yo * rowe, rowe * int64_t(sizeof(R)));
        const uint32_t tb = uint32_t(st * 24 * kTile) * uint32_t(sizeof(R));
        const int pl = lane >> 4, col = (lane & 15) * 4;   // 4 planes of 64 words per instruction
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int p = 4 * j + pl;
            const u32x4 v = *(const u32x4*)&sh.lam[b][p][lc + col];
            row_store16(rl, on ? tb + uint32_t(p * kTile + col) * 4u : kNoStore, v);
        }
        if constexpr (GRAD) {
            const __amdgpu_buffer_rsrc_t rg = row_rsrc(gsum + yo * rowg, rowg * 4);
            const u32x4 v = *(const u32x4*)&sh.gs[b][pl][lc + col];
            row_store16(rg, on ? uint32_t(st * 4 * kTile + pl * kTile + col) * 4u : kNoStore, v);
        }
    };
    // mu, lam of the rows of the levels, newest first
    float prm[NT][2];
#pragma unroll
    for (int t = 0; t < NT; ++t) prm[t][0] = prm[t][1] = 0.0f;

    // lambda of levels t = 0 .. NT-2 of the rows behind: q3 of the last two rows, q0 and q2 of
    // the last row shifted to the lanes that pull them
    R hq3a[NT - 1][6], hq3b[NT - 1][6], ho0[NT - 1][6], ho2[NT - 1][6];
#pragma unroll
    for (int t = 0; t < NT - 1; ++t)
#pragma unroll
        for (int k = 0; k < 6; ++k) hq3a[t][k] = hq3b[t][k] = ho0[t][k] = ho2[t][k] = R(0);
    // the lane that owns its column for the direct FP64 updates: on a grid narrower than the
    // span, columns beyond nx wrap onto nodes other lanes own
    const bool own_col = out_lane && c0 + pos < nx;

    const int iters = Sy + 2 * (NT - 1);
    // a window that starts past the last stored tile: barriers only (see march_kernel)
    if (c0 + ws >= ntile * kTile) {
        for (int i = 0; i < iters; ++i) __syncthreads();
        return;
    }
    prefetch_row(rw[0], rw[1], rw[2]);
#pragma unroll
    for (int t = 0; t < NT; ++t) prefetch_level(t, rw[t + 1]);
    store_row(rw[NT], false, 0);
    // The first 2 (NT - 1) iterations, in which levels are still starting, are peeled off
    // the steady loop, which then needs no checks for them (a compile-time flag).
    auto iteration = [&](int i, auto steady_c) {
        constexpr bool steady = decltype(steady_c)::value;
        R f[4][6];
        R l[4][6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            l[0][k] = pre[k];
            l[1][k] = pre[6 + k];
            l[2][k] = pre[12 + k];
            l[3][k] = pre[18 + k];
        }
        if constexpr (FIELDS) {
#pragma unroll
            for (int t = NT - 1; t >= 1; --t) {
                prm[t][0] = prm[t - 1][0];
                prm[t][1] = prm[t - 1][1];
            }
            prm[0][0] = pprm[0];
            prm[0][1] = pprm[1];
        }

        // ring slot of the row of level t: the iteration in which its first level ran, mod NT
        const int slot0 = i % NT;
        float gn[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        auto level = [&](int t, int y, R out[4][6]) {
            R mu, lam;
            if (FIELDS && cm.mu) mu = prm[t][0]; else mu = kval<R>(cm.mu0, cm.f_mu0);
            if (FIELDS && cm.lam) lam = prm[t][1]; else lam = kval<R>(cm.lam0, cm.f_lam0);
            R inc[4];
            adj_node<R, LAW>(cm, l, prec[t], mu, lam, R(a.r[t]), gpar, gbody, out, inc);
            const bool probe = (pmw[t] >> (xc & 31)) & 1u;
            const int64_t idx = int64_t(y) * nx + xc;
            double ps[2] = {0.0, 0.0};
            if (probe) {
                ps[0] = a.probe_weight * a.pfield[idx];
                ps[1] = a.probe_weight * a.pfield[n + idx];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    out[q][0] += R(ps[0]);
                    out[q][1] += R(ps[1]);
                }
            }
            if constexpr (GRAD) {
                const int slot = slot0 - t < 0 ? slot0 - t + NT : slot0 - t;
                if (t == 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) gn[j] = pgs[j];
                } else {
                    const float4 v = sh.ring[slot][w][lane];
                    gn[0] = v.x; gn[1] = v.y; gn[2] = v.z; gn[3] = v.w;
                }
                // the row of level t is an output row of the segment
                const bool own = own_col && (steady || i >= NT - 1 + t) && i < Sy + NT - 1 + t;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (!has[j]) continue;
                    gn[j] = gn[j] + float(inc[j]);
                    if (a.fold[t]) {
                        // One lane owns each node and at most one level of a pass folds
                        // (levels <= 4 < kGradBlock), so a return-less FP64 atomic add at
                        // L2 performs the same addition as a load, add and store, without
                        // the wave waiting for the load.  At a probe node the body gradient
                        // also takes the probe term below by load and store, so both of its
                        // updates stay plain there: every address sees one kind of access.
                        if (own) {
                            if (j >= 2 && probe)
                                g64[j][idx] += double(gn[j]);
                            else
                                __hip_atomic_fetch_add(g64[j] + idx, double(gn[j]), __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                        }
                        gn[j] = 0.0f;
                    }
                }
                if (own && probe && gbody) {
                    a.g_body[idx] += a.r[t] * hdt * ps[0];
                    a.g_body[n + idx] += a.r[t] * hdt * ps[1];
                }
                if (t < NT - 1) sh.ring[slot][w][lane] = make_float4(gn[0], gn[1], gn[2], gn[3]);
            }
        };
        level(0, rw[1], f);
        // every load is issued on every iteration, whether its level runs or not, so that the
        // memory operations in flight are the same on all paths through the loop
        prefetch_row(wrap_inc(rw[0], ny), rw[0], rw[1]);
        prefetch_level(0, rw[0]);
#pragma unroll
        for (int L = 2; L <= NT; ++L) {
            const bool started = steady || i >= 2 * (L - 2);  // level L-2 of the pass has run
            const bool act = steady || i >= 2 * (L - 1);
            if (act) {
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    l[0][k] = ho0[L - 2][k];
                    l[1][k] = f[1][k];
                    l[2][k] = ho2[L - 2][k];
                    l[3][k] = hq3b[L - 2][k];
                }
            }
            if (started) {
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    hq3b[L - 2][k] = hq3a[L - 2][k];
                    hq3a[L - 2][k] = f[3][k];
                    ho0[L - 2][k] = from_next(f[0][k]);
                    ho2[L - 2][k] = from_prev(f[2][k]);
                }
            }
            if (act) level(L - 1, rw[L], f);
            prefetch_level(L - 1, rw[L - 1]);
        }
        // f, gn: lambda and the block sums of the pass's last level at output row
        // y1 - (NT - 1) from iteration 2 (NT - 1) on
        const bool outp = steady || i >= 2 * (NT - 1);
        const int b = i & 1;
        if (outp && out_lane) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < 6; ++k) sh.lam[b][6 * q + k][pos] = f[q][k];
            if constexpr (GRAD) {
#pragma unroll
                for (int j = 0; j < 4; ++j) sh.gs[b][j][pos] = gn[j];
            }
        }
        __syncthreads();
        store_row(rw[NT], outp, b);
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
}

// ---------------------------------------------------------------- dispatch

template <int ST, int LAW, bool FIELDS, bool GRAD>
static hipError_t march_adj_levels(const MarchAdjArgs& a, hipStream_t s) {
    const dim3 grid(unsigned(a.nwg)), block(kMarchWaves * kTile);
    switch (a.levels) {
        case 2: hipLaunchKernelGGL((march_adj_kernel<ST, LAW, FIELDS, 2, GRAD>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((march_adj_kernel<ST, LAW, FIELDS, 3, GRAD>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((march_adj_kernel<ST, LAW, FIELDS, 4, GRAD>), grid, block, 0, s, a); break;
    }
    return hipGetLastError();
}

template <int ST, int LAW>
static hipError_t march_adj_st_law(const MarchAdjArgs& a, hipStream_t s) {
    const bool fields = a.cm.mu || a.cm.lam;
    const bool grad = a.g_mu || a.g_lam || a.g_body;
    if (fields) return grad ? march_adj_levels<ST, LAW, true, true>(a, s) : march_adj_levels<ST, LAW, true, false>(a, s);
    return grad ? march_adj_levels<ST, LAW, false, true>(a, s) : march_adj_levels<ST, LAW, false, false>(a, s);
}

template <int ST>
static hipError_t march_adj_st(const MarchAdjArgs& a, hipStream_t s) {
    switch (a.cm.material) {
        case LBM_LOGNH: return march_adj_st_law<ST, LBM_LOGNH>(a, s);
        case LBM_NH: return march_adj_st_law<ST, LBM_NH>(a, s);
        case LBM_MR: return march_adj_st_law<ST, LBM_MR>(a, s);
        case LBM_YEOH: return march_adj_st_law<ST, LBM_YEOH>(a, s);
        case LBM_GENT: return march_adj_st_law<ST, LBM_GENT>(a, s);
        default: return march_adj_st_law<ST, LBM_SVK>(a, s);
    }
}

// FP32 and FP16 storage share the kernel: the adjoint populations and the records are in
// the FP32 compute type for both.
hipError_t launch_march_adjoint(const MarchAdjArgs& a, hipStream_t s) { return march_adj_st<LBM_F32_SHIFTED>(a, s); }

}  // namespace lbm
