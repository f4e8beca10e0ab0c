// C ABI of the library (declared in include/lbm.h): argument validation, buffer sizes and
// the launch sequence of each entry point.  No allocation, no synchronisation.
#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "lbm_device.hpp"
#include "lbm_internal.hpp"

using namespace lbm;

namespace {

// Device scratch of lbm_diagnostics_noalloc: the per-workgroup partial sums of the
// diagnostics reduction, kDiagBlocks x LBM_DIAG_COUNT doubles (80 KiB), enough for every
// grid because the reduction kernel strides over the nodes with at most kDiagBlocks
// workgroups.  Every GPU the library runs on holds its own copy until the process ends.
// On the host this name is only a stand-in for the symbol: host code uses the device
// address that scratch_address obtains for the current device.
__device__ __align__(256) double scratch[kDiagBlocks * LBM_DIAG_COUNT];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
lbm_status scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LBM_ERR_LAUNCH;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_ERR_LAUNCH;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

bool any_wall(const lbm_params* p) {
    for (int e = 0; e < 4; ++e)
        if (p->bc[e] != LBM_PERIODIC) return true;
    return false;
}

bool has_traction(const lbm_params* p) {
    for (int e = 0; e < 4; ++e)
        if (p->bc[e] == LBM_TRACTION) return true;
    return false;
}

size_t real_size(const lbm_params* p) { return p->storage == LBM_F64_PLAIN ? 8 : 4; }

size_t pop_elem_size(const lbm_params* p) {
    return p->storage == LBM_F64_PLAIN ? 8 : (p->storage == LBM_F16_SHIFTED ? 2 : 4);
}

Common make_common(const lbm_params* p, const lbm_state* s) {
    Common cm{};
    cm.nx = p->nx;
    cm.ny = p->ny;
    cm.ntile = (p->nx + kTile - 1) / kTile;
    for (int e = 0; e < 4; ++e) cm.bc[e] = p->bc[e];
    cm.periodic_x = p->bc[LBM_XMIN] == LBM_PERIODIC;
    cm.periodic_y = p->bc[LBM_YMIN] == LBM_PERIODIC;
    cm.material = p->material;
    cm.storage = p->storage;
    cm.dx = p->dx;
    cm.c = p->c;
    cm.omega = p->omega;
    cm.dt = p->dx / p->c;
    cm.newton_max_iter = p->newton_max_iter > 0 ? p->newton_max_iter : 8;
    cm.newton_tol = p->newton_tol > 0 ? p->newton_tol : (p->storage == LBM_F64_PLAIN ? 1e-14 : 1e-6);
    for (int k = 0; k < 3; ++k) cm.law_k[k] = p->law_k[k];
    cm.k_omq = 0.25 * cm.omega;
    cm.k_cq = 0.5 * cm.omega / cm.c;
    cm.k_srcw = cm.dt * (2.0 - cm.omega) * 0.125;
    cm.k_hdt = 0.5 * cm.dt;
    cm.k_c2 = 2.0 / cm.c;
    cm.k_hc = 0.5 / cm.c;
    if (s) {
        cm.mu0 = s->mu0;
        cm.lam0 = s->lam0;
        cm.b0[0] = s->b0[0];
        cm.b0[1] = s->b0[1];
        cm.mu = s->mu;
        cm.lam = s->lam;
        cm.body = s->body;
        cm.body_prev = s->body_prev;
        cm.fault = s->fault;
    }
    cm.f_omq = float(cm.k_omq);
    cm.f_cq = float(cm.k_cq);
    cm.f_srcw = float(cm.k_srcw);
    cm.f_hdt = float(cm.k_hdt);
    cm.f_c2 = float(cm.k_c2);
    cm.f_hc = float(cm.k_hc);
    cm.f_dt = float(cm.dt);
    cm.f_mu0 = float(cm.mu0);
    cm.f_lam0 = float(cm.lam0);
    for (int k = 0; k < 3; ++k) cm.f_law_k[k] = float(cm.law_k[k]);
    cm.f_omega = float(cm.omega);
    return cm;
}

EdgeData make_edges(const lbm_edge_data* ed) {
    EdgeData out{};
    if (ed) {
        for (int e = 0; e < 4; ++e) {
            out.value[e][0] = ed->value[e][0];
            out.value[e][1] = ed->value[e][1];
            out.field[e] = ed->field[e];
        }
    }
    return out;
}

lbm_status check_state(const lbm_params* p, const lbm_state* s, bool need_ustar = true) {
    if (!s || !s->pop[0] || !s->pop[1] || !s->fault) return LBM_ERR_ARG;
    if (need_ustar && !s->ustar) return LBM_ERR_ARG;
    if (s->cur != 0 && s->cur != 1) return LBM_ERR_ARG;
    if (has_traction(p) && !s->aux) return LBM_ERR_ARG;
    return LBM_OK;
}

lbm_status launched(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_ERR_LAUNCH; }

// Uniform predeformation: I when none is given; rejected unless finite with det > 0.
bool predeformation(const double* Fbar, double out[4]) {
    const double I[4] = {1.0, 0.0, 0.0, 1.0};
    const double* f = Fbar ? Fbar : I;
    for (int k = 0; k < 4; ++k) {
        if (!isfinite(f[k])) return false;
        out[k] = f[k];
    }
    return out[0] * out[3] - out[1] * out[2] > 0.0;
}

// The P-wave speed at F = I bounding the material's waves: sqrt(lam + 2 mu) for the
// Lame-parametrised laws, sqrt(lam + 4 G / 3) for the invariant laws (small-strain shear
// modulus G, plane Lame constant lam - 2 G / 3).
double p_wave_speed(const lbm_params* p, double mu_max, double lam_max) {
    double cp2 = lam_max + 2.0 * mu_max;
    if (p->material == LBM_MR || p->material == LBM_YEOH || p->material == LBM_GENT) {
        const double G = p->material == LBM_MR ? 2.0 * (p->law_k[0] + p->law_k[1]) * mu_max
                       : p->material == LBM_YEOH ? 2.0 * p->law_k[0] * mu_max : mu_max;
        cp2 = lam_max + 4.0 / 3.0 * G;
    }
    return sqrt(fmax(cp2, 0.0));
}

// Growth per step of the modes a traction wall carries at omega = 2, measured (FP64, 512^2,
// from noise; walls on all four sides, with a velocity corner, and on two sides only) at
// P-wave ratios c_p / c of 0.0505 ... 0.283, and the rate at which 2 - omega damps them.
constexpr int kWallTable = 6;
constexpr double kWallRatio[kWallTable] = {0.0505, 0.0707, 0.101, 0.141, 0.202, 0.283};
constexpr double kWallGrowth0[kWallTable] = {3.3e-4, 2.7e-4, 2.5e-4, 3.7e-4, 1.76e-3, 4.35e-3};
constexpr double kWallDamping = 0.45;
constexpr double kWallGrowthMax = 2e-4;   // e-folding in 5000 steps

}  // namespace

extern "C" {

size_t lbm_tile_width(void) { return (size_t)kTile; }

size_t lbm_padded_nodes(const lbm_params* p) {
    const size_t ntile = ((size_t)p->nx + kTile - 1) / kTile;
    return ntile * kTile * (size_t)p->ny;
}

size_t lbm_pop_bytes(const lbm_params* p) { return 24 * lbm_padded_nodes(p) * pop_elem_size(p); }

size_t lbm_ustar_bytes(const lbm_params* p) {
    // FP64: 2 double planes; shifted storages: 2 float planes S and 2 double planes U
    return p->storage == LBM_F64_PLAIN ? 2 * lbm_padded_nodes(p) * 8 : lbm_padded_nodes(p) * (2 * 4 + 2 * 8);
}

// F^b of every link (4 values), and for the two-level step the wall lines of level n+1
// (2 lines of 24 values per link) and U^{n+1} of the wall nodes (6 values), 8 bytes each
// (WallLines in lbm_kernel_util.hpp).
size_t lbm_aux_bytes(const lbm_params* p) { return (size_t)(2 * p->nx + 2 * p->ny) * (4 + 2 * 24 + 6) * 8; }

size_t lbm_record_bytes(const lbm_params* p) { return 6 * lbm_padded_nodes(p) * real_size(p); }

size_t lbm_adj_bytes(const lbm_params* p) { return 24 * lbm_padded_nodes(p) * real_size(p); }

size_t lbm_adj_sum_bytes(const lbm_params* p) { return 4 * lbm_padded_nodes(p) * sizeof(float); }

size_t lbm_diag_scratch_bytes(const lbm_params* p) {
    (void)p;
    return (size_t)kDiagBlocks * LBM_DIAG_COUNT * sizeof(double);
}

lbm_status lbm_check_params(const lbm_params* p) {
    if (!p) return LBM_ERR_ARG;
    if (p->nx < 3 || p->ny < 3) return LBM_ERR_ARG;
    if ((int64_t)p->nx * (int64_t)p->ny >= ((int64_t)1 << 31)) return LBM_ERR_ARG;
    if (p->material < LBM_LOGNH || p->material > LBM_GENT) return LBM_ERR_ARG;
    if (p->material == LBM_MR &&
        !(p->law_k[0] >= 0 && p->law_k[1] >= 0 && p->law_k[0] + p->law_k[1] > 0)) return LBM_ERR_ARG;
    if (p->material == LBM_YEOH &&
        !(p->law_k[0] > 0 && isfinite(p->law_k[1]) && isfinite(p->law_k[2]))) return LBM_ERR_ARG;
    if (p->material == LBM_GENT && !(p->law_k[0] > 0 && isfinite(p->law_k[0]))) return LBM_ERR_ARG;
    if (p->storage < LBM_F32_SHIFTED || p->storage > LBM_F64_PLAIN) return LBM_ERR_ARG;
    for (int e = 0; e < 4; ++e)
        if (p->bc[e] < LBM_PERIODIC || p->bc[e] > LBM_TRACTION) return LBM_ERR_ARG;
    if ((p->bc[LBM_XMIN] == LBM_PERIODIC) != (p->bc[LBM_XMAX] == LBM_PERIODIC)) return LBM_ERR_ARG;
    if ((p->bc[LBM_YMIN] == LBM_PERIODIC) != (p->bc[LBM_YMAX] == LBM_PERIODIC)) return LBM_ERR_ARG;
    if (any_wall(p) && (p->nx < 4 || p->ny < 4)) return LBM_ERR_ARG;
    if (!(p->dx > 0) || !(p->c > 0) || !(p->omega > 0) || !(p->omega <= 2.0)) return LBM_ERR_ARG;
    return LBM_OK;
}

double lbm_wall_mode_growth(const lbm_params* p, double mu_max, double lam_max) {
    if (!p || !(p->c > 0)) return 0.0;
    bool traction = false;
    for (int e = 0; e < 4; ++e) traction |= p->bc[e] == LBM_TRACTION;
    if (!traction) return 0.0;
    const double r = p_wave_speed(p, mu_max, lam_max) / p->c;
    double g0;
    if (r <= kWallRatio[0]) {
        g0 = kWallGrowth0[0];
    } else {
        int i = 1;
        while (i < kWallTable - 1 && r > kWallRatio[i]) ++i;
        // linear between the measured points, and along the last segment beyond them
        const double t = (r - kWallRatio[i - 1]) / (kWallRatio[i] - kWallRatio[i - 1]);
        g0 = kWallGrowth0[i - 1] + t * (kWallGrowth0[i] - kWallGrowth0[i - 1]);
    }
    return g0 - kWallDamping * (2.0 - p->omega);
}

lbm_status lbm_check_cfl(const lbm_params* p, double mu_max, double lam_max) {
    if (!p || !(p->c > 0)) return LBM_ERR_ARG;
    if (p_wave_speed(p, mu_max, lam_max) / p->c > 0.5) return LBM_ERR_CFL;
    if (lbm_wall_mode_growth(p, mu_max, lam_max) > kWallGrowthMax) return LBM_ERR_CFL;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_params* p, lbm_state* s, const double* v0, const double* u0,
                    const double* Fbar, double r0, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if ((st = check_state(p, s)) != LBM_OK) return st;
    if (!v0) return LBM_ERR_ARG;
    double F0[4];
    if (!predeformation(Fbar, F0)) return LBM_ERR_ARG;
    if (!p->force_unstable) {
        const double mu = s->mu ? s->mu_max : s->mu0;
        const double lam = s->lam ? s->lam_max : s->lam0;
        if ((st = lbm_check_cfl(p, mu, lam)) != LBM_OK) return st;
    }
    InitArgs a{};
    a.cm = make_common(p, s);
    a.v0 = v0;
    a.u0 = u0;
    for (int k = 0; k < 4; ++k) a.Fbar[k] = F0[k];
    a.r0 = r0;
    a.scratch = s->pop[1 - s->cur];
    a.dst = s->pop[s->cur];
    a.ustar = s->ustar;
    return launched(launch_init(a, (hipStream_t)stream));
}

lbm_status lbm_init_state(const lbm_params* p, lbm_state* s, const double* U0, const double* dUdX,
                          const double* dUdY, const double* u0, double r0, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if ((st = check_state(p, s)) != LBM_OK) return st;
    if (!U0 || !dUdX || !dUdY) return LBM_ERR_ARG;
    if (!p->force_unstable) {
        const double mu = s->mu ? s->mu_max : s->mu0;
        const double lam = s->lam ? s->lam_max : s->lam0;
        if ((st = lbm_check_cfl(p, mu, lam)) != LBM_OK) return st;
    }
    InitArgs a{};
    a.cm = make_common(p, s);
    a.v0 = U0;                       // planes 0, 1 of U0 are v0
    a.u0 = u0;
    a.r0 = r0;
    a.scratch = const_cast<double*>(U0);
    a.dst = s->pop[s->cur];
    a.ustar = s->ustar;
    a.dUdX = dUdX;
    a.dUdY = dUdY;
    return launched(launch_init_given(a, (hipStream_t)stream));
}

lbm_status lbm_step(const lbm_params* p, lbm_state* s, int64_t n, double r_n, double r_np1,
                    const lbm_edge_data* at_half, void* record, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if ((st = check_state(p, s, false)) != LBM_OK) return st;
    if (any_wall(p) && !at_half) return LBM_ERR_ARG;
    const hipStream_t hs = (hipStream_t)stream;
    const Common cm = make_common(p, s);
    const EdgeData ed = make_edges(at_half);
    {
        TractionArgs t{};
        t.cm = cm;
        if (cm.body_prev) t.cm.body = cm.body_prev;
        t.pop = s->pop[s->cur];
        t.aux = s->aux;
        t.r_n = r_n;
        t.ed = ed;
        if (launch_traction(t, hs) != hipSuccess) return LBM_ERR_LAUNCH;
    }
    StepArgs a{};
    a.cm = cm;
    a.src = s->pop[s->cur];
    a.dst = s->pop[1 - s->cur];
    a.ustar = s->ustar;
    a.aux = s->aux;
    a.record = record;
    a.fold = (n + 1) % kUstarBlock == 0;
    a.r_np1 = r_np1;
    a.ed = ed;
    if (launch_step(a, hs) != hipSuccess) return LBM_ERR_LAUNCH;
    s->cur = 1 - s->cur;
    return LBM_OK;
}

lbm_status lbm_step2(const lbm_params* p, lbm_state* s, int64_t n, double r_n, double r_np1, double r_np2,
                     const lbm_edge_data* at_half, const lbm_edge_data* at_half_next, void* record1, void* record2,
                     void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if ((st = check_state(p, s, false)) != LBM_OK) return st;
    const bool walls = any_wall(p);
    if (walls && (!at_half || !at_half_next || !s->aux)) return LBM_ERR_ARG;
    const hipStream_t hs = (hipStream_t)stream;
    Step2Args a{};
    a.cm = make_common(p, s);
    a.cm.body_prev = nullptr;                    // the body field is that of every level
    a.src = s->pop[s->cur];
    a.dst = s->pop[1 - s->cur];
    a.ustar = s->ustar;
    a.aux = s->aux;
    a.ed = make_edges(at_half);
    a.ed2 = make_edges(at_half_next);
    a.record1 = record1;
    a.record2 = record2;
    a.fold1 = (n + 1) % kUstarBlock == 0;
    a.fold2 = (n + 2) % kUstarBlock == 0;
    a.nstrip = (p->nx + kPairCols - 1) / kPairCols;
    a.r_np1 = r_np1;
    a.r_np2 = r_np2;
    for (int k = 0; k < 2; ++k) {
        a.fb1[k] = float(r_np1 * a.cm.b0[k]);
        a.fb2[k] = float(r_np2 * a.cm.b0[k]);
    }
    // F^b of level n from f*^n, as lbm_step takes it
    {
        TractionArgs t{};
        t.cm = a.cm;
        t.pop = a.src;
        t.aux = s->aux;
        t.r_n = r_n;
        t.ed = a.ed;
        if (launch_traction(t, hs) != hipSuccess) return LBM_ERR_LAUNCH;
    }
    if (launch_step2(a, hs) != hipSuccess) return LBM_ERR_LAUNCH;
    if (walls) {
        // F^b of level n+1 from the wall lines the bulk kernel wrote, then the wall nodes
        {
            TractionArgs t{};
            t.cm = a.cm;
            t.pop = nullptr;
            t.aux = s->aux;
            t.r_n = r_np1;
            t.ed = a.ed2;
            t.lines = 1;
            if (launch_traction(t, hs) != hipSuccess) return LBM_ERR_LAUNCH;
        }
        Step2Args w = a;
        w.wall_pass = 1;
        if (launch_step2(w, hs) != hipSuccess) return LBM_ERR_LAUNCH;
    }
    s->cur = 1 - s->cur;
    return LBM_OK;
}

// Compute units of the current device, queried once per device (256 on an MI355X).
static int compute_units() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev].store(v, std::memory_order_relaxed);
    return v;
}

// Workgroups of the multi-level kernels: spans of kMarchTiles tiles per row, segments of
// `seg` rows.  A segment repeats 2 (levels - 1) rows of the first level and fewer of the
// later ones, and the launch runs in rounds of one workgroup per compute unit: the length
// between 8 and 1024 rows that minimises rounds x iterations per workgroup (8192^2: 205
// rows in three full rounds; with at most 64 rows, 62 rows in ten rounds ran 4 % slower).
static bool march_geometry(const lbm_params* p, int levels, int& nspan, int& seg, int& nwg, FastDiv& d_nspan) {
    const int ntile = (p->nx + kTile - 1) / kTile;
    nspan = (ntile + kMarchTiles - 1) / kMarchTiles;
    const int cus = compute_units();
    int best = 8;
    int64_t best_cost = -1;
    for (int sg = 8; sg <= 1024; ++sg) {
        const int64_t ns = (p->ny + sg - 1) / sg;
        const int64_t rounds = (ns * nspan + cus - 1) / cus;
        const int64_t cost = rounds * (sg + 2 * (levels - 1));
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = sg; }
    }
    seg = best < p->ny ? best : p->ny;
    const int64_t nseg = (p->ny + seg - 1) / seg;
    if (nseg * nspan > 0x7fffffff) return false;
    nwg = int(nseg * nspan);
    d_nspan = fast_div(nspan);
    return true;
}

lbm_status lbm_step_multi(const lbm_params* p, lbm_state* s, int64_t n, int levels, const double* r_next,
                          void* const* records, int record_planes, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if ((st = check_state(p, s, false)) != LBM_OK) return st;
    if (levels < 2 || levels > kMarchMaxLevels || !r_next) return LBM_ERR_ARG;
    if (records) {
        for (int t = 0; t < levels; ++t)
            if (!records[t]) return LBM_ERR_ARG;
        if (record_planes != 6 && record_planes != 4) return LBM_ERR_ARG;
    } else if (!s->ustar) {
        return LBM_ERR_ARG;
    }
    if (any_wall(p)) return LBM_ERR_UNSUPPORTED;
    // the replay form: records, no accumulator, shifted storages
    if (records && (s->ustar || p->storage == LBM_F64_PLAIN)) return LBM_ERR_UNSUPPORTED;
    MarchArgs a{};
    a.cm = make_common(p, s);
    a.cm.body_prev = nullptr;
    a.src = s->pop[s->cur];
    a.dst = s->pop[1 - s->cur];
    a.ustar = s->ustar;
    a.levels = levels;
    a.rec_planes = records ? record_planes : 6;
    for (int t = 0; t < levels; ++t) {
        a.fold[t] = (n + 1 + t) % kUstarBlock == 0;
        a.rec[t] = records ? records[t] : nullptr;
        a.r[t] = r_next[t];
        for (int k = 0; k < 2; ++k) a.fb[t][k] = float(r_next[t] * a.cm.b0[k]);
    }
    if (!march_geometry(p, levels, a.nspan, a.seg, a.nwg, a.d_nspan)) return LBM_ERR_UNSUPPORTED;
    if (launch_march(a, (hipStream_t)stream) != hipSuccess) return LBM_ERR_LAUNCH;
    s->cur = 1 - s->cur;
    return LBM_OK;
}

static lbm_status recover_common(const lbm_params* p, const lbm_state* s, double r_n, void* out,
                                 RecoverArgs& a, bool need_ustar = false) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if ((st = check_state(p, s, need_ustar)) != LBM_OK) return st;
    if (!out) return LBM_ERR_ARG;
    a = RecoverArgs{};
    a.cm = make_common(p, s);
    a.pop = s->pop[s->cur];
    a.ustar = s->ustar;
    a.r_n = r_n;
    a.out = out;
    return LBM_OK;
}

lbm_status lbm_displacement(const lbm_params* p, const lbm_state* s, double r_n, double* u_out, void* stream) {
    RecoverArgs a;
    lbm_status st = recover_common(p, s, r_n, u_out, a, true);
    if (st != LBM_OK) return st;
    return launched(launch_displacement(a, (hipStream_t)stream));
}

lbm_status lbm_moments(const lbm_params* p, const lbm_state* s, double r_n, double* U_out, void* stream) {
    RecoverArgs a;
    lbm_status st = recover_common(p, s, r_n, U_out, a);
    if (st != LBM_OK) return st;
    return launched(launch_moments(a, (hipStream_t)stream));
}

lbm_status lbm_record_state(const lbm_params* p, const lbm_state* s, double r_n, void* record, void* stream) {
    RecoverArgs a;
    lbm_status st = recover_common(p, s, r_n, record, a);
    if (st != LBM_OK) return st;
    return launched(launch_record(a, (hipStream_t)stream));
}

lbm_status lbm_stress(const lbm_params* p, const lbm_state* s, double r_n, double* P_out, double* sigma_out,
                      void* stream) {
    RecoverArgs a;
    lbm_status st = recover_common(p, s, r_n, P_out, a);
    if (st != LBM_OK) return st;
    a.out2 = sigma_out;
    return launched(launch_stress(a, (hipStream_t)stream));
}

lbm_status lbm_diagnostics(const lbm_params* p, const lbm_state* s, double r_n, double* out, void* scratch,
                           void* stream) {
    RecoverArgs a;
    lbm_status st = recover_common(p, s, r_n, out, a);
    if (st != LBM_OK) return st;
    if (!scratch) return LBM_ERR_ARG;
    a.scratch = scratch;
    return launched(launch_diagnostics(a, (hipStream_t)stream));
}

lbm_status lbm_diagnostics_noalloc(const lbm_params* p, const lbm_state* s, double r_n, double* out,
                                   void* stream) {
    if (p && lbm_diag_scratch_bytes(p) > sizeof(scratch)) return LBM_ERR_UNSUPPORTED;
    void* ptr = nullptr;
    const lbm_status st = scratch_address(&ptr);
    if (st != LBM_OK) return st;
    return lbm_diagnostics(p, s, r_n, out, ptr, stream);
}

lbm_status lbm_adjoint_step(const lbm_params* p, const lbm_state* fwd, lbm_adj_state* adj, int64_t m,
                            double r_m, const lbm_edge_data* at_half, const void* record_m, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if (!fwd || !adj || !adj->adj[0] || !adj->adj[1] || !record_m) return LBM_ERR_ARG;
    if (adj->cur != 0 && adj->cur != 1) return LBM_ERR_ARG;
    if (has_traction(p) && !adj->aux) return LBM_ERR_ARG;
    if (adj->nprobe < 0 || (adj->nprobe > 0 && (!adj->probe || !adj->ubar))) return LBM_ERR_ARG;
    if (m < 0 || m > adj->nsteps) return LBM_ERR_ARG;
    if (any_wall(p) && !at_half) return LBM_ERR_ARG;
    if (p->storage != LBM_F64_PLAIN && (adj->g_mu || adj->g_lam || adj->g_body) && !adj->gsum)
        return LBM_ERR_ARG;
    AdjArgs a{};
    a.cm = make_common(p, fwd);
    a.src = adj->adj[adj->cur];
    a.dst = adj->adj[1 - adj->cur];
    a.record = record_m;
    a.g_mu = adj->g_mu;
    a.g_lam = adj->g_lam;
    a.g_body = adj->g_body;
    a.gsum = adj->gsum;
    a.fold = m % kGradBlock == 0;
    a.aux = adj->aux;
    a.r_m = r_m;
    a.ed = make_edges(at_half);
    a.probe = adj->probe;
    a.ubar = adj->ubar;
    a.nprobe = adj->nprobe;
    a.probe_weight = (m == adj->nsteps ? 0.5 : 1.0) * a.cm.dt;
    if (adj->nprobe > 0 && adj->probe_mask && adj->probe_field) {
        a.pmask = adj->probe_mask;
        a.pfield = adj->probe_field;
    }
    if (launch_adjoint(a, (hipStream_t)stream) != hipSuccess) return LBM_ERR_LAUNCH;
    adj->cur = 1 - adj->cur;
    return LBM_OK;
}

size_t lbm_probe_mask_bytes(const lbm_params* p) {
    if (lbm_check_params(p) != LBM_OK) return 0;
    return size_t((p->nx + kTile - 1) / kTile) * size_t(p->ny) * sizeof(uint64_t);
}

lbm_status lbm_adjoint_probe_table(const lbm_params* p, const lbm_adj_state* adj, uint64_t* mask, double* field,
                                   void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if (!adj || !mask || !field) return LBM_ERR_ARG;
    if (adj->nprobe < 0 || (adj->nprobe > 0 && (!adj->probe || !adj->ubar))) return LBM_ERR_ARG;
    const Common cm = make_common(p, nullptr);
    return launched(launch_probe_table(cm, adj->probe, adj->ubar, adj->nprobe, mask, field, (hipStream_t)stream));
}

lbm_status lbm_adjoint_step2(const lbm_params* p, const lbm_state* fwd, lbm_adj_state* adj, int64_t m, double r_m,
                             double r_mm1, const lbm_edge_data* at_half, const lbm_edge_data* at_half_prev,
                             const void* record_m, const void* record_mm1, const uint64_t* mask,
                             const double* field, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if (!fwd || !adj || !adj->adj[0] || !adj->adj[1] || !record_m || !record_mm1) return LBM_ERR_ARG;
    if (any_wall(p) && (!at_half || !at_half_prev || !adj->aux)) return LBM_ERR_ARG;
    if (adj->cur != 0 && adj->cur != 1) return LBM_ERR_ARG;
    if (adj->nprobe < 0 || (adj->nprobe > 0 && (!adj->probe || !adj->ubar || !mask || !field))) return LBM_ERR_ARG;
    if (m < 1 || m >= adj->nsteps) return LBM_ERR_ARG;
    if (p->storage != LBM_F64_PLAIN && (adj->g_mu || adj->g_lam || adj->g_body) && !adj->gsum)
        return LBM_ERR_ARG;
    Adj2Args a{};
    a.cm = make_common(p, fwd);
    a.src = adj->adj[adj->cur];
    a.dst = adj->adj[1 - adj->cur];
    a.rec1 = record_m;
    a.rec2 = record_mm1;
    a.g_mu = adj->g_mu;
    a.g_lam = adj->g_lam;
    a.g_body = adj->g_body;
    a.gsum = adj->gsum;
    a.fold1 = m % kGradBlock == 0;
    a.fold2 = (m - 1) % kGradBlock == 0;
    a.nstrip = (p->nx + kTile - 1) / kTile;
    {
        const int nblk = (p->ny + kPairRows - 1) / kPairRows;
        a.map = pair_map(a.nstrip, nblk, 0, a.nstrip, 0, nblk);
    }
    a.r1 = r_m;
    a.r2 = r_mm1;
    a.pmask = adj->nprobe > 0 ? mask : nullptr;
    a.pfield = adj->nprobe > 0 ? field : nullptr;
    a.probe_weight = a.cm.dt;                    // levels m and m - 1 are below N
    a.aux = adj->aux;
    if (any_wall(p)) {
        a.ed1 = make_edges(at_half);
        a.ed2 = make_edges(at_half_prev);
    }
    if (launch_adjoint2(a, (hipStream_t)stream) != hipSuccess) return LBM_ERR_LAUNCH;
    adj->cur = 1 - adj->cur;
    return LBM_OK;
}

lbm_status lbm_adjoint_step_multi(const lbm_params* p, const lbm_state* fwd, lbm_adj_state* adj, int64_t m,
                                  int levels, const double* r, const void* const* records, const uint64_t* mask,
                                  const double* field, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if (!fwd || !adj || !adj->adj[0] || !adj->adj[1] || !r || !records) return LBM_ERR_ARG;
    if (levels < 2 || levels > kMarchMaxLevels) return LBM_ERR_ARG;
    if (adj->cur != 0 && adj->cur != 1) return LBM_ERR_ARG;
    if (adj->nprobe < 0 || (adj->nprobe > 0 && (!adj->probe || !adj->ubar || !mask || !field))) return LBM_ERR_ARG;
    if (m - (levels - 1) < 0 || m >= adj->nsteps) return LBM_ERR_ARG;
    for (int t = 0; t < levels; ++t)
        if (!records[t]) return LBM_ERR_ARG;
    if (any_wall(p) || p->storage == LBM_F64_PLAIN) return LBM_ERR_UNSUPPORTED;
    if ((adj->g_mu || adj->g_lam || adj->g_body) && !adj->gsum) return LBM_ERR_ARG;
    MarchAdjArgs a{};
    a.cm = make_common(p, fwd);
    a.src = adj->adj[adj->cur];
    a.dst = adj->adj[1 - adj->cur];
    for (int t = 0; t < levels; ++t) {
        a.rec[t] = records[t];
        a.r[t] = r[t];
        a.fold[t] = (m - t) % kGradBlock == 0;
    }
    a.g_mu = adj->g_mu;
    a.g_lam = adj->g_lam;
    a.g_body = adj->g_body;
    a.gsum = adj->gsum;
    a.pmask = adj->nprobe > 0 ? mask : nullptr;
    a.pfield = adj->nprobe > 0 ? field : nullptr;
    a.probe_weight = a.cm.dt;                    // every level of the pass is below N
    a.levels = levels;
    if (!march_geometry(p, levels, a.nspan, a.seg, a.nwg, a.d_nspan)) return LBM_ERR_UNSUPPORTED;
    if (launch_march_adjoint(a, (hipStream_t)stream) != hipSuccess) return LBM_ERR_LAUNCH;
    adj->cur = 1 - adj->cur;
    return LBM_OK;
}

lbm_status lbm_adjoint_init(const lbm_params* p, const lbm_state* fwd, lbm_adj_state* adj, const double* v0,
                            const double* u0, const double* Fbar, double r0, double* g_v0, void* stream) {
    lbm_status st = lbm_check_params(p);
    if (st != LBM_OK) return st;
    if (!fwd || !adj || !adj->adj[0] || !adj->adj[1] || !v0 || !g_v0) return LBM_ERR_ARG;
    double F0[4];
    if (!predeformation(Fbar, F0)) return LBM_ERR_ARG;
    if (adj->cur != 0 && adj->cur != 1) return LBM_ERR_ARG;
    if (adj->nprobe < 0 || (adj->nprobe > 0 && (!adj->probe || !adj->ubar))) return LBM_ERR_ARG;
    AdjInitArgs a{};
    a.cm = make_common(p, fwd);
    a.lam0 = adj->adj[adj->cur];
    a.scratch = adj->adj[1 - adj->cur];
    a.v0 = v0;
    a.u0 = u0;
    for (int k = 0; k < 4; ++k) a.Fbar[k] = F0[k];
    a.r0 = r0;
    a.g_mu = adj->g_mu;
    a.g_lam = adj->g_lam;
    a.g_body = adj->g_body;
    a.g_v0 = g_v0;
    a.probe = adj->probe;
    a.ubar = adj->ubar;
    a.nprobe = adj->nprobe;
    return launched(launch_adjoint_init(a, (hipStream_t)stream));
}

const char* lbm_status_string(lbm_status st) {
    switch (st) {
        case LBM_OK: return "ok";
        case LBM_ERR_ARG: return "invalid argument";
        case LBM_ERR_UNSUPPORTED: return "unsupported combination";
        case LBM_ERR_CFL: return "lattice speed too low for the material (bulk: P-wave speed above c/2; traction walls: wall modes grow, see lbm_wall_mode_growth)";
        case LBM_ERR_LAUNCH: return "kernel launch failed";
        default: return "unknown status";
    }
}

const char* lbm_version(void) { return "tlvlbm 0.1 (gfx950)"; }

}  // extern "C"
