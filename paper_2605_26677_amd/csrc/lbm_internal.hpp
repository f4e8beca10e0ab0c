// Internal launch interface between the C-ABI layer (lbm_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

constexpr int kBlock = 256;          // threads per workgroup of the node-indexed kernels
constexpr int kTilesPerBlock = 2;    // 64-node tiles (one wavefront each) per workgroup of the
                                     // step and adjoint kernels
constexpr int kDiagBlocks = 1024;    // partial sums of the diagnostics reduction
constexpr int kTracWin = 64;         // wall links one wavefront of the traction solve takes

// Offsets of each edge's links in the traction staging buffer (links, not bytes).
__host__ __device__ inline void edge_offsets(int nx, int ny, int off[4], int len[4]) {
    len[LBM_XMIN] = ny; len[LBM_XMAX] = ny; len[LBM_YMIN] = nx; len[LBM_YMAX] = nx;
    off[LBM_XMIN] = 0; off[LBM_XMAX] = ny; off[LBM_YMIN] = 2 * ny; off[LBM_YMAX] = 2 * ny + nx;
}

// The same for one edge, without an array: where e differs between the lanes of a
// wavefront, an array indexed by e would be placed in scratch memory.
__host__ __device__ inline int edge_off(int nx, int ny, int e) {
    return e == LBM_XMIN ? 0 : e == LBM_XMAX ? ny : e == LBM_YMIN ? 2 * ny : 2 * ny + nx;
}
__host__ __device__ inline int edge_len(int nx, int ny, int e) {
    return (e == LBM_XMIN || e == LBM_XMAX) ? ny : nx;
}

struct EdgeData {
    double value[4][2];
    const double* field[4];
};

struct Common {
    int nx, ny;
    int ntile;                       // tiles of kTile nodes per row
    int bc[4];
    int periodic_x, periodic_y;
    int material, storage;
    double dx, c, omega, dt;
    double mu0, lam0, b0[2];
    const float* mu;
    const float* lam;
    const float* body;
    const float* body_prev;          // field of level n for the step n -> n+1 (or NULL)
    uint32_t* fault;
    int newton_max_iter;
    double newton_tol;
    double law_k[3];                 // invariant-law constants (lbm_params.law_k)
    // collision constants, formed once on the host: omega/4, omega/(2c), the forcing weight
    // dt (2 - omega)/8 of eq:collision, and dt/2
    double k_omq, k_cq, k_srcw, k_hdt;
    double k_c2, k_hc;               // 2/c and 1/(2c) (adjoint)
    // The same constants, dt, the uniform mu, lam and the law constants rounded to float
    // on the host, for the FP32 compute type: a float kernel argument enters an
    // instruction as a scalar operand, while converting the double costs a vector
    // instruction per wavefront and use.  kval() picks the copy of the compute type.
    float f_omq, f_cq, f_srcw, f_hdt, f_c2, f_hc, f_dt, f_mu0, f_lam0, f_law_k[3], f_omega;
};

// A Common constant in the compute type R: the float copy for R = float (the same value
// as converting the double on the device), the double otherwise.
template <typename R>
__host__ __device__ __forceinline__ R kval(double d, float f) {
    if constexpr (sizeof(R) == sizeof(float)) return f;
    else return R(d);
}

struct StepArgs {
    Common cm;
    const void* src;                 // f*^n
    void* dst;                       // f*^{n+1}
    void* ustar;
    const void* aux;                 // F^b per traction link (compute type, 4 per link)
    void* record;                    // U^{n+1} or NULL
    int fold;                        // shifted storages: move S into U this step (ustar_refs)
    double r_np1;
    EdgeData ed;                     // data at t^{n+1/2}
};

// Two fused steps (step2_kernel, adjoint2_kernel): workgroups of kPairWaves row wavefronts
// and one edge wavefront, each owning kPairRows rows of a strip of kPairCols (one tile of)
// columns.
constexpr int kPairWaves = 7;
constexpr int kPairRows = kPairWaves - 2;
constexpr int kPairCols = 64;
constexpr int kPairChunk = 32;       // strips per chunk of the workgroup order

// Workgroups of a two-level launch.  mode 0: the blocks [s_lo, s_hi) x [b_lo, b_hi) of
// strips x block rows, in chunks of `chunk` strips side by side and inside a chunk one
// block row after the other (per_chunk = chunk * (b_hi - b_lo) workgroups per chunk), so
// that the workgroups that re-read a block's edge rows run soon after it on the same
// XCD's L2.  mode 1: every block outside that rectangle (the blocks along the walls):
// block rows [0, b_lo) and [b_hi, nblk) over all strips, then the strips outside
// [s_lo, s_hi) over the block rows [b_lo, b_hi).
// Division of 0 <= v < 2^31 by a divisor d >= 1 fixed per launch, by multiplication
// (Granlund and Montgomery, division by invariant integers): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, v / d = (mulhi(m, v) + v) >> l.  The host forms m and l;
// on the device both steps are scalar instructions for a wave-uniform v, where a plain
// integer division would take a vector reciprocal sequence.
struct FastDiv {
    uint32_t m;
    int l;
    int d;
};

inline FastDiv fast_div(int d) {
    FastDiv f{};
    f.d = d < 1 ? 1 : d;
    int l = 0;
    while ((int64_t(1) << l) < f.d) ++l;
    f.l = l;
    f.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - uint64_t(f.d))) / uint64_t(f.d) + 1);
    return f;
}

__device__ __forceinline__ int fdiv(int v, const FastDiv& f) {
    const uint32_t t = __umulhi(f.m, uint32_t(v));
    return int((t + uint32_t(v)) >> f.l);
}

struct PairMap {
    int mode;
    int nstrip, nblk;
    int s_lo, s_hi, b_lo, b_hi;
    int chunk, per_chunk;
    FastDiv d_per_chunk, d_chunk, d_last;    // mode 0: divisions by per_chunk, by chunk and
                                             // by the width of the last (narrower) chunk
};

// Workgroups of mode 0 over the given rectangle; the chunk width is kPairChunk strips,
// fewer where chunk * rows would not fit 32-bit arithmetic.
inline PairMap pair_map(int nstrip, int nblk, int s_lo, int s_hi, int b_lo, int b_hi) {
    PairMap m{};
    m.mode = 0;
    m.nstrip = nstrip;
    m.nblk = nblk;
    m.s_lo = s_lo; m.s_hi = s_hi; m.b_lo = b_lo; m.b_hi = b_hi;
    const int64_t rows = b_hi - b_lo;
    int64_t c = kPairChunk;
    while (c > 1 && c * rows > 0x7fffffff) c >>= 1;
    if (c > s_hi - s_lo) c = s_hi - s_lo;
    if (c < 1) c = 1;
    m.chunk = int(c);
    m.per_chunk = int(c * rows);
    m.d_per_chunk = fast_div(m.per_chunk);
    m.d_chunk = fast_div(m.chunk);
    const int width = s_hi - s_lo, last = width - (width - 1) / m.chunk * m.chunk;
    m.d_last = fast_div(last);
    return m;
}

inline int64_t pair_map_blocks(const PairMap& m) {
    const int64_t inner = int64_t(m.s_hi - m.s_lo) * (m.b_hi - m.b_lo);
    return m.mode == 0 ? inner : int64_t(m.nstrip) * m.nblk - inner;
}

__device__ __forceinline__ void pair_block(const PairMap& m, int b, int& strip, int& blk) {
    if (m.mode == 0) {
        const int chunk = fdiv(b, m.d_per_chunk);
        const int rem = b - chunk * m.per_chunk;
        const int kc = min(m.chunk, (m.s_hi - m.s_lo) - chunk * m.chunk);
        const int bb = kc == m.chunk ? fdiv(rem, m.d_chunk) : fdiv(rem, m.d_last);
        strip = m.s_lo + chunk * m.chunk + (rem - bb * kc);
        blk = m.b_lo + bb;
        return;
    }
    const int n1 = m.b_lo * m.nstrip, n2 = (m.nblk - m.b_hi) * m.nstrip;
    if (b < n1) {
        blk = b / m.nstrip;
        strip = b - blk * m.nstrip;
    } else if (b < n1 + n2) {
        const int j = b - n1;
        blk = m.b_hi + j / m.nstrip;
        strip = j % m.nstrip;
    } else {
        const int side = m.s_lo + (m.nstrip - m.s_hi);
        const int j = b - n1 - n2;
        blk = m.b_lo + j / side;
        const int t = j % side;
        strip = t < m.s_lo ? t : m.s_hi + (t - m.s_lo);
    }
}

struct Step2Args {
    Common cm;
    const void* src;                 // f*^n
    void* dst;                       // f*^{n+2}
    void* ustar;
    void* aux;                       // F^b staging and wall lines (grids with walls)
    EdgeData ed;                     // wall data at t^{n+1/2}
    EdgeData ed2;                    // wall data at t^{n+3/2}
    float fb1[2], fb2[2];            // uniform body r_np1 b0 and r_np2 b0 rounded to float
    int wall_pass;                   // launch the wall-node kernel instead of the bulk kernel
    void* record1;                   // U^{n+1} or NULL
    void* record2;                   // U^{n+2} or NULL
    int fold1, fold2;                // accumulator folds after the first / second step
    int nstrip;                      // strips of kPairCols columns (= tiles per row)
    PairMap map;                     // the workgroups of this launch (the interior ones
                                     // of a split launch)
    PairMap map2;                    // split launch: the rim workgroups (wall code)
    int n_rim, rim_period;           // split launch: rim workgroups, one every rim_period
    FastDiv d_rim_period;
    double r_np1, r_np2;
};

// Several levels per pass on periodic grids (march_kernel): workgroups of kMarchWaves
// wavefronts, each workgroup owning a span of kMarchTiles aligned tiles and a segment of
// `seg` rows.
constexpr int kMarchMaxLevels = 4;
constexpr int kMarchWaves = 8;
constexpr int kMarchTiles = 7;
constexpr int kMarchSpan = kMarchTiles * 64;

struct MarchArgs {
    Common cm;
    const void* src;                 // f*^n
    void* dst;                       // f*^{n+levels}
    void* ustar;
    int levels;                      // 2 .. kMarchMaxLevels
    int fold[kMarchMaxLevels];       // accumulator fold after level n+1+t
    double r[kMarchMaxLevels];       // body factor r(n+1+t)
    float fb[kMarchMaxLevels][2];    // uniform body r(n+1+t) b0 rounded to float
    void* rec[kMarchMaxLevels];      // records of U^{n+1+t} (the replay form), or NULL
    int rec_planes;                  // 6: whole records; 4: the F - I planes 2 .. 5 only
    int nspan, seg, nwg;             // spans per row, rows per segment, workgroups
    FastDiv d_nspan;
};

// Several adjoint levels per pass on periodic grids (march_adj_kernel), the same workgroups
// as march_kernel.
struct MarchAdjArgs {
    Common cm;
    const void* src;                 // lambda^{m+1}
    void* dst;                       // lambda^{m+1-levels}
    const void* rec[kMarchMaxLevels];   // U^{m-t}, t = 0 .. levels - 1
    double r[kMarchMaxLevels];       // body factors r(m - t)
    int fold[kMarchMaxLevels];       // block-sum fold at level m - t
    double* g_mu;
    double* g_lam;
    double* g_body;
    void* gsum;
    const uint64_t* pmask;           // probe table (lbm_adjoint_probe_table) or NULL
    const double* pfield;
    double probe_weight;
    int levels;
    int nspan, seg, nwg;
    FastDiv d_nspan;
};

struct TractionArgs {
    Common cm;
    const void* pop;                 // f*^n
    void* aux;
    double r_n;
    EdgeData ed;
    int eblk[5];                     // workgroups of edge e: [eblk[e], eblk[e+1]) (0 for non-traction)
    int lines;                       // read level n from the wall lines of aux instead of pop
};

struct RecoverArgs {
    Common cm;
    const void* pop;
    const void* ustar;
    double r_n;
    void* out;                       // double planes (moments / displacement) or record
    void* out2;                      // second output (Cauchy stress) or NULL
    void* scratch;                   // diagnostics partials
};

struct InitArgs {
    Common cm;
    const double* v0;
    const double* u0;
    double Fbar[4];                  // uniform predeformation (I when none is given)
    double r0;
    void* scratch;                   // U0 as 6 double planes (stride n)
    void* dst;                       // f*^0
    void* ustar;
    const double* dUdX;              // derivatives of U0 (6 double planes each) given by the
    const double* dUdY;              // caller, or NULL: finite differences of U0
};

struct AdjArgs {
    Common cm;
    const void* src;                 // lambda^{m+1}
    void* dst;                       // lambda^m
    const void* record;              // U^m
    double* g_mu;
    double* g_lam;
    double* g_body;
    void* gsum;                      // FP32 block sums of the gradients (4 tiled planes)
    int fold;                        // move the block sums into the FP64 gradients
    void* aux;
    double r_m;
    EdgeData ed;
    int eblk[5];                     // traction stage 1: workgroups of edge e, [eblk[e], eblk[e+1])
    int sblk[5];                     // traction stage 2: the same for the scatter
    const int32_t* probe;
    const double* ubar;
    int nprobe;
    double probe_weight;             // dt * (1 or 1/2)
    const uint64_t* pmask;           // probe table (mask, summed ubar field) or NULL
    const double* pfield;
    int lines;                       // traction stage 1: lambda^{m+1} of the wall nodes from
                                     // the staged wall lines of aux instead of src
};

struct Adj2Args {
    Common cm;
    const void* src;                 // lambda^{m+1}
    void* dst;                       // lambda^{m-1}
    const void* rec1;                // U^m
    const void* rec2;                // U^{m-1}
    double* g_mu;
    double* g_lam;
    double* g_body;
    void* gsum;
    int fold1, fold2;                // block-sum folds at levels m and m - 1
    int nstrip;
    PairMap map;                     // as in Step2Args
    double r1, r2;                   // body factors r(m), r(m-1)
    const uint64_t* pmask;           // probe table (lbm_adjoint_probe_table) or NULL
    const double* pfield;
    double probe_weight;             // weight of level m's probe source
    void* aux;                       // grids with walls: traction staging and wall lines
    EdgeData ed1, ed2;               // wall data at t^{m+1/2} and t^{m-1/2}
};

struct AdjInitArgs {
    Common cm;
    const void* lam0;                // lambda^0
    void* scratch;                   // 12 double planes: U0 (6) and the v0 seeds (6)
    const double* v0;
    const double* u0;
    double Fbar[4];
    double r0;
    double* g_mu;
    double* g_lam;
    double* g_body;
    double* g_v0;
    const int32_t* probe;
    const double* ubar;
    int nprobe;
};

hipError_t launch_step(const StepArgs& a, hipStream_t s);
hipError_t launch_step2(const Step2Args& a, hipStream_t s);
hipError_t launch_march(const MarchArgs& a, hipStream_t s);
hipError_t launch_march_adjoint(const MarchAdjArgs& a, hipStream_t s);
hipError_t launch_traction(TractionArgs a, hipStream_t s);   // every traction edge, one launch
hipError_t launch_moments(const RecoverArgs& a, hipStream_t s);
hipError_t launch_record(const RecoverArgs& a, hipStream_t s);
hipError_t launch_displacement(const RecoverArgs& a, hipStream_t s);
hipError_t launch_diagnostics(const RecoverArgs& a, hipStream_t s);
hipError_t launch_stress(const RecoverArgs& a, hipStream_t s);
hipError_t launch_init(const InitArgs& a, hipStream_t s);
hipError_t launch_init_given(const InitArgs& a, hipStream_t s);
hipError_t launch_init_state(const InitArgs& a, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& a, hipStream_t s);
hipError_t launch_adjoint_init(const AdjInitArgs& a, hipStream_t s);
hipError_t launch_adjoint2(const Adj2Args& a, hipStream_t s);
hipError_t launch_probe_table(const Common& cm, const int32_t* probe, const double* ubar, int nprobe,
                              uint64_t* mask, double* field, hipStream_t s);

}  // namespace lbm
