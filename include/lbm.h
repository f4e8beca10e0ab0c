/*
 * lbm.h - C ABI of the MI355X library for the total-Lagrangian vectorial lattice
 * Boltzmann method (D2Q4 lattice, six-component vector populations) of Feng & Chu,
 * "A total-Lagrangian vectorial lattice Boltzmann method for finite-strain hyperelastic
 * dynamics", arXiv 2605.26677.  Section, equation and table names below are the paper's.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer named "device" is a device pointer on the current HIP device, owned by
 *    the caller.  The library never allocates, frees or synchronises: each call only
 *    enqueues kernels on `stream` (a hipStream_t passed as void*; NULL = null stream) and
 *    returns.  Argument errors are returned synchronously as lbm_status codes, launch
 *    errors as LBM_ERR_LAUNCH; numerical faults found on the device are OR-ed into the
 *    caller's fault word (LBM_FAULT_*) without stopping the stream.
 *  - Grid: nx x ny nodes; node (a, b) sits at X = ((a + 1/2) dx, (b + 1/2) dx), so the
 *    half-way walls of Sec. 3.6 lie at X = 0, X = nx dx, Y = 0, Y = ny dx.  Time step
 *    dt = dx / c (Sec. 2.1: c = dx/dt is the nondimensional lattice speed).
 *  - Field planes: a "plane" is nx*ny values, row-major (index b*nx + a).  Arrays of
 *    several planes place plane k at offset k*nx*ny unless stated otherwise.
 *  - Tiled arrays: populations, the u* accumulator and state records are stored in tiles
 *    of W = lbm_tile_width() (= 64) consecutive nodes of one row, each tile holding all of
 *    its planes contiguously: element (p, a, b) of an array of NP planes is at index
 *    ((b * T + a / W) * NP + p) * W + a % W, T = ceil(nx / W) tiles per row
 *    (lbm_padded_nodes() = T * W * ny nodes, padding nodes unused).
 *  - Population buffers: NP = 24 planes, p = 6*q + k; q is the D2Q4 direction in the
 *    paper's order (1,0), (0,1), (-1,0), (0,-1) (Sec. 3.1), k the component of
 *    U = (v1, v2, F11, F12, F21, F22) (eq:state-vector).  A buffer holds post-collision
 *    populations f* (eq:collision) of one time level; for the shifted storages it holds
 *    g* = f* - (0, 0, 1/4, 0, 0, 1/4), i.e. F is carried as F - I (the equilibrium of the
 *    reference state U = (0, 0, 1, 0, 0, 1) is U/4, because P(I) = 0 for every law of
 *    Appendix A).
 *  - Time levels: after lbm_init the state holds f*^0 and the displacement accumulator
 *    u*^1; lbm_step advances f*^n to f*^{n+1} (streaming, half-way wall rules with data at
 *    t^{n+1/2}, moments at level n+1, collision) and u*^{n+1} to u*^{n+2}.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
enum {
    LBM_OK = 0,
    LBM_ERR_ARG = 1,          /* invalid argument (sizes, enums, NULL pointers, pairing) */
    LBM_ERR_UNSUPPORTED = 2,  /* combination not provided by the library */
    LBM_ERR_CFL = 3,          /* lattice speed too low for the material (see lbm_check_cfl) */
    LBM_ERR_LAUNCH = 4        /* a kernel launch failed (hipGetLastError) */
};

/* Population storage.  F32/F16 carry F - I and compute in FP32; F64 stores the plain
 * (unshifted) populations and computes in FP64. */
enum { LBM_F32_SHIFTED = 0, LBM_F16_SHIFTED = 1, LBM_F64_PLAIN = 2 };

/* Hyperelastic closures of Appendix A: logarithmic neo-Hookean (eq:lognh-model,
 * P = mu (F - F^-T) + lam ln J F^-T), compressible neo-Hookean (eq:nh-model,
 * P = mu (F - F^-T) + lam/2 (J^2 - 1) F^-T), St. Venant-Kirchhoff (eq:svk-model), and the
 * invariant-based Mooney-Rivlin (eq:mr-model), Yeoh (eq:yeoh-model) and Gent
 * (eq:gent-model) laws in the plane-strain modified invariants of eq:modified-invariants,
 * each with the bulk term lam/2 (ln J)^2.  The invariant laws take their constants from
 * lbm_params.law_k as multiples of mu, so that P stays linear in (mu, lam) over a
 * heterogeneous mu field:
 *   LBM_MR:   law_k = (c10/mu, c01/mu, unused)   (Appendix A's default: c10 + c01 = mu/2)
 *   LBM_YEOH: law_k = (c1/mu, c2/mu, c3/mu)      (Appendix A's default: c1 = mu/2)
 *   LBM_GENT: law_k = (J_m, unused, unused); a state with barI1 - 3 >= J_m is
 *             inadmissible and is reported like J <= 0.
 * Their small-strain shear modulus is 2 (c10 + c01), 2 c1 and mu respectively, and their
 * small-strain plane Lame constant is lam - 2/3 of that shear modulus. */
enum { LBM_LOGNH = 0, LBM_NH = 1, LBM_SVK = 2, LBM_MR = 3, LBM_YEOH = 4, LBM_GENT = 5 };

/* Edge kinds: periodic, velocity Dirichlet (eq:dirichlet-boundary-rule), nominal-traction
 * Neumann (eq:neumann-boundary-rule).  Periodic edges must pair: XMIN with XMAX, YMIN
 * with YMAX. */
enum { LBM_PERIODIC = 0, LBM_VELOCITY = 1, LBM_TRACTION = 2 };
enum { LBM_XMIN = 0, LBM_XMAX = 1, LBM_YMIN = 2, LBM_YMAX = 3 };

/* Bits of the device fault word. */
enum {
    LBM_FAULT_J = 1,          /* inadmissible state at some node: det F <= 0 (Sec. 2.2), or
                                 barI1 - 3 >= J_m for the Gent law (Appendix A) */
    LBM_FAULT_NONFINITE = 2,  /* a recovered state value is not finite */
    LBM_FAULT_NEWTON = 4,     /* a traction-boundary Newton solve failed (Sec. 3.6) */
    LBM_FAULT_PROBE = 8       /* an adjoint kernel met a probe index outside [0, nx*ny) and
                                 skipped it (the gradients then miss that probe's term) */
};

/* Number of FP64 values written by lbm_diagnostics. */
#define LBM_DIAG_COUNT 10

typedef struct {
    int32_t nx, ny;            /* grid nodes, >= 4 along any axis with walls, >= 3 otherwise */
    int32_t material;          /* LBM_LOGNH | LBM_NH | LBM_SVK | LBM_MR | LBM_YEOH | LBM_GENT */
    int32_t storage;           /* LBM_F32_SHIFTED | LBM_F16_SHIFTED | LBM_F64_PLAIN */
    int32_t bc[4];             /* per edge LBM_XMIN..LBM_YMAX: LBM_PERIODIC | LBM_VELOCITY | LBM_TRACTION */
    int32_t newton_max_iter;   /* traction Newton updates per link; <= 0 selects 8 */
    int32_t force_unstable;    /* nonzero: skip the lattice-speed audit */
    double dx;                 /* lattice spacing (> 0) */
    double c;                  /* lattice speed dx/dt (> 0) */
    double omega;              /* BGK rate, 0 < omega <= 2 (eq:collision; 2 is nondissipative) */
    double newton_tol;         /* relative Newton tolerance; <= 0 selects 1e-14 (F64) or 1e-6 (F32/F16) */
    double law_k[3];           /* constants of the invariant-based laws (see LBM_MR); ignored
                                  by the others.  MR: both >= 0 with a positive sum; Yeoh:
                                  c1/mu > 0; Gent: J_m > 0 */
} lbm_params;

typedef struct {
    void *pop[2];              /* device: two population buffers of lbm_pop_bytes() each */
    int32_t cur;               /* index of the buffer that holds the current level */
    void *ustar;               /* device, lbm_ustar_bytes(): u* of eq:trapezoid-u, tiled;
                                  F64: 2 double planes.  F32/F16: u* = U + S with S 2 float
                                  planes (tiled, first) and U 2 double planes (tiled, after
                                  S): each step adds dt v to S, and the step n -> n+1 with
                                  (n + 1) % 16 == 0 moves S into U, so S never sums more
                                  than 16 increments in FP32 (n should count levels).  May
                                  be NULL for lbm_step (the quadrature is then skipped, as
                                  in a replay for the adjoint) but not for lbm_init or
                                  lbm_displacement */
    const float *mu, *lam;     /* device: per-node Lame fields (1 plane each), or NULL for mu0/lam0 */
    double mu0, lam0;          /* uniform values used when the field pointer is NULL */
    double mu_max, lam_max;    /* host-known upper bounds of the fields (CFL audit);
                                  ignored when the field pointer is NULL */
    const float *body;         /* device: body acceleration b, 2 planes, or NULL for b0; the
                                  force at level m is r(m) b (the r factors are per call) */
    const float *body_prev;    /* device, optional: body field of the previous level for
                                  lbm_step (level n of the step n -> n+1, read where the step
                                  recovers the state of level n: traction walls); NULL means
                                  the same field as body.  Lets a caller drive a force that is
                                  not a fixed field times a ramp by swapping two buffers. */
    double b0[2];              /* uniform body acceleration when body is NULL */
    void *aux;                 /* device, lbm_aux_bytes(): wall staging (F^b per traction link;
                                  level n+1 on the wall lines for lbm_step2) */
    uint32_t *fault;           /* device: fault word (LBM_FAULT_* bits are OR-ed in) */
} lbm_state;

/* Boundary data at t^{n+1/2} (eq:boundary-general): for velocity edges the prescribed
 * velocity v_D, for traction edges the nominal traction T (force per reference length,
 * eq:neumann-continuum).  value[e] is uniform along edge e unless field[e] is non-NULL:
 * then field[e] is a device array of 2*L doubles (component-major, L = ny for x-edges,
 * nx for y-edges, position along the edge = a or b). */
typedef struct {
    double value[4][2];
    const double *field[4];
} lbm_edge_data;

/* ------------------------------------------------------------------ sizes */

/* Nodes per tile of the tiled arrays (64). */
size_t lbm_tile_width(void);
/* Nodes of a tiled array including row padding: ceil(nx / 64) * 64 * ny. */
size_t lbm_padded_nodes(const lbm_params *p);
/* Bytes of one population buffer: 24 * lbm_padded_nodes() * element size. */
size_t lbm_pop_bytes(const lbm_params *p);
/* Bytes of the u* accumulator. */
size_t lbm_ustar_bytes(const lbm_params *p);
/* Bytes of the wall staging buffer (forward and adjoint): F^b of every link, and for
 * lbm_step2 level n+1 on the wall line and first interior line of every edge. */
size_t lbm_aux_bytes(const lbm_params *p);
/* Bytes of one per-level state record (6 tiled planes of the compute type: v1, v2, F - I). */
size_t lbm_record_bytes(const lbm_params *p);
/* Bytes of device scratch needed by lbm_diagnostics. */
size_t lbm_diag_scratch_bytes(const lbm_params *p);

/* ------------------------------------------------------------------ checks */

/* Validates p.  Returns LBM_ERR_ARG or LBM_ERR_UNSUPPORTED on bad input, else LBM_OK. */
lbm_status lbm_check_params(const lbm_params *p);

/* Lattice-speed audit (Sec. 4 audits c against the largest tangent wave speed, Table
 * tab:validation-setup): at F = I the fastest wave is the P wave, sqrt(lam + 2 mu) for the
 * Lame-parametrised laws and sqrt(lam + 4/3 G) for the invariant laws with small-strain
 * shear modulus G.  Returns LBM_ERR_CFL
 *   - when that speed exceeds c/2: the linearised D2Q4 x 6 step is then unstable in the
 *     bulk at omega = 2 (periodic grids);
 *   - on a grid with a traction edge, when lbm_wall_mode_growth exceeds 2e-4 per step (an
 *     e-folding within 5000 steps): traction walls carry modes confined to the wall line
 *     and its corners that grow at omega = 2 at a rate set by c_p / c and independent of
 *     the grid size, so they need 2 - omega > 0 to be damped;
 * and LBM_OK otherwise.  Finite strains can raise the tangent speeds (lbm_diagnostics out[9]
 * audits the current state).  lbm_init runs this audit unless force_unstable, which short
 * runs near omega = 2 (the manufactured solutions of Sec. 4.2) set. */
lbm_status lbm_check_cfl(const lbm_params *p, double mu_max, double lam_max);

/* Estimated growth per step of the traction-wall modes (0 without a traction edge): a
 * measured growth at omega = 2 as a function of c_p / c (linear between the measured ratios
 * 0.05 ... 0.28 and beyond them along the last segment), minus 0.45 (2 - omega), the damping
 * the BGK rate gives them.  A negative value means the modes decay. */
double lbm_wall_mode_growth(const lbm_params *p, double mu_max, double lam_max);

/* ------------------------------------------------------------------ forward */

/* Second-order population initialisation (Sec. 3.4, eq:init-compact, eq:init-Zq-components,
 * eq:init-deltaPq, eq:init-expanded), computed in FP64 with second-order finite
 * differences (one-sided next to non-periodic walls) and rounded to the storage type;
 * then the first collision (eq:collision at level 0) so that s->pop[s->cur] holds f*^0,
 * and u*^1 = u0 - (dt/2) v0 + dt v^0 (eq:trapezoid-u).
 *   v0: device, 2 double planes, initial velocity.
 *   u0: device, 2 double planes, initial displacement, or NULL for 0.
 *   Fbar: host, 4 doubles (F11, F12, F21, F22) of a uniform predeformation, or NULL for I:
 *     the initial deformation gradient is Fbar + grad u0 (Sec. 5.2 starts waves on a
 *     homogeneous finite state).  The affine part (Fbar - I) X of the displacement is not
 *     carried in u*: lbm_displacement returns the part that starts from u0.
 *   r0: factor applied to the body force at t = 0 (B^0 = r0 b).
 * Uses s->pop[1 - s->cur] as scratch.  Runs the CFL audit unless force_unstable. */
lbm_status lbm_init(const lbm_params *p, lbm_state *s, const double *v0, const double *u0,
                    const double *Fbar, double r0, void *stream);

/* The second-order initialisation of lbm_init from a state and its spatial derivatives that
 * the caller gives (for fields known in closed form, as the manufactured solutions of
 * Sec. 4, whose runs start from the exact derivatives), then the same first collision and
 * u*^1 = u0 - (dt/2) v0 + dt v^0.
 *   U0: device, 6 double planes (v1, v2, F11 - 1, F12, F21, F22 - 1).
 *   dUdX, dUdY: device, 6 double planes each, the X and Y derivatives of those components.
 *   u0: device, 2 double planes, initial displacement, or NULL for 0.
 *   r0: factor applied to the body force at t = 0.
 * s->pop[1 - s->cur] is not touched.  Runs the CFL audit unless force_unstable. */
lbm_status lbm_init_state(const lbm_params *p, lbm_state *s, const double *U0, const double *dUdX,
                          const double *dUdY, const double *u0, double r0, void *stream);

/* One time step (Sec. 3.7), level n -> n+1, fused in one pass over the grid: pull
 * streaming (eq:streaming) from s->pop[s->cur], half-way reconstruction of every missing
 * link with the data at t^{n+1/2} (eq:boundary-general; traction links first solve for
 * F^b, Sec. 3.6), moments with B^{n+1} = r_np1 b (eq:moment-U), P(F) in registers,
 * equilibrium (eq:feq), collision with trapezoidal forcing (eq:collision), store into
 * s->pop[1 - s->cur], u* update.  Flips s->cur on success.
 *   r_n, r_np1: body-force factors at levels n and n+1.
 *   at_half: boundary data at t^{n+1/2}; may be NULL only when all edges are periodic
 *     (LBM_ERR_ARG otherwise).
 *   record: device, lbm_record_bytes(), receives U^{n+1} (v, F - I), or NULL. */
lbm_status lbm_step(const lbm_params *p, lbm_state *s, int64_t n, double r_n, double r_np1,
                    const lbm_edge_data *at_half, void *record, void *stream);

/* Two time steps, level n -> n+2, in one pass over the grid (temporal blocking of the
 * step of Sec. 3.7: level n+1 stays on chip).  The result, the u* accumulator, the records
 * and the fault bits are those of lbm_step(n) followed by lbm_step(n+1), bit for bit, at
 * about half the HBM traffic per level.  Flips s->cur on success.
 *   r_n, r_np1, r_np2: body-force factors at levels n, n+1, n+2.  The body field s->body (or
 *     the uniform b0) is that of every level: s->body_prev is not read.
 *   at_half, at_half_next: boundary data at t^{n+1/2} and t^{n+3/2}; may be NULL only when
 *     all edges are periodic (LBM_ERR_ARG otherwise).
 *   record1, record2: device, lbm_record_bytes() each, receive U^{n+1} and U^{n+2} (v,
 *     F - I) as lbm_step's record would; either may be NULL.
 * On a grid with walls the bulk pass also leaves level n+1 of the wall lines and the first
 * interior lines in s->aux; the traction F^b of level n+1 is solved from them and a small
 * pass completes the wall nodes (s->aux must hold lbm_aux_bytes()). */
lbm_status lbm_step2(const lbm_params *p, lbm_state *s, int64_t n, double r_n, double r_np1,
                     double r_np2, const lbm_edge_data *at_half, const lbm_edge_data *at_half_next,
                     void *record1, void *record2, void *stream);

/* `levels` time steps (2 to 4), level n -> n+levels, in one pass over a periodic grid
 * (temporal blocking of the step of Sec. 3.7; the levels in between stay in registers).
 * The result, the u* accumulator, the records and the fault bits are those of `levels`
 * calls of lbm_step, bit for bit on every node, at about 1/levels of the HBM traffic per
 * level; the padding nodes of the tiled arrays (beyond nx in a row's last tile) receive
 * unspecified values, which no entry point reads.  Flips s->cur on success.
 *   r_next: host array of `levels` body-force factors r(n+1) ... r(n+levels).  The body
 *     field s->body (or the uniform b0) is that of every level: s->body_prev is not read.
 *   records: NULL, or a host array of `levels` device pointers that receive U^{n+1} ...
 *     U^{n+levels} (lbm_record_bytes() each) as lbm_step's record would: the replay of the
 *     checkpointed adjoint, which requires s->ustar = NULL (the accumulator is not
 *     updated) and F32 or F16 storage (LBM_ERR_UNSUPPORTED otherwise).
 *   record_planes: with records, 6 writes whole records; 4 writes only the F - I planes
 *     (2 .. 5), all that the adjoint entry points read, and leaves the velocity planes of
 *     the records as they were (a third fewer record bytes).  Ignored without records.
 * Without records s->ustar must be set.  Returns LBM_ERR_ARG when levels is outside
 * [2, 4], r_next or a record pointer is NULL, record_planes is neither 6 nor 4 with
 * records, or s->ustar is NULL without records, and
 * LBM_ERR_UNSUPPORTED on a grid with a wall (lbm_step2 takes those). */
lbm_status lbm_step_multi(const lbm_params *p, lbm_state *s, int64_t n, int levels,
                          const double *r_next, void *const *records, int record_planes,
                          void *stream);

/* Displacement at the current level n (eq:trapezoid-u): u^n = u*^{n+1} - (dt/2) v^n with
 * v^n recovered from the stored post-collision populations (sum_q f* = U + (dt/2) B).
 *   r_n: body-force factor at level n.  u_out: device, 2 double planes. */
lbm_status lbm_displacement(const lbm_params *p, const lbm_state *s, double r_n, double *u_out,
                            void *stream);

/* State U^n = (v1, v2, F11-1, F12, F21, F22-1) of the current level, recovered from the
 * stored populations.  U_out: device, 6 double planes. */
lbm_status lbm_moments(const lbm_params *p, const lbm_state *s, double r_n, double *U_out,
                       void *stream);

/* Stress recovery at the current level (Sec. 3.5): first Piola stress P(F) of the
 * selected law and Cauchy stress sigma = J^{-1} P F^T.  P_out: device, 4 double planes
 * (P11, P12, P21, P22); sigma_out: device, 3 double planes (s11, s12, s22), or NULL. */
lbm_status lbm_stress(const lbm_params *p, const lbm_state *s, double r_n, double *P_out,
                      double *sigma_out, void *stream);

/* FP64 reductions over the current level: out[0..1] sum of v, out[2..5] sum of F - I,
 * out[6] energy sum(|v|^2/2 + W(F)) dx^2, out[7] min J, out[8] max |F - I| (Frobenius),
 * out[9] max over nodes of the P-wave-bound ratio sqrt(lam_max(Q(n;F)))/c with the
 * acoustic tensor of eq:acoustic-tensor-section2 scanned over 180 directions.
 *   out: device, LBM_DIAG_COUNT doubles.  scratch: device, lbm_diag_scratch_bytes(). */
lbm_status lbm_diagnostics(const lbm_params *p, const lbm_state *s, double r_n, double *out,
                           void *scratch, void *stream);

/* lbm_diagnostics for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same kernels and result,
 * bit for bit, with the reduction's partial sums in a fixed 80 KiB device array of the
 * library instead of caller scratch.  Allocates nothing; the array's device address is
 * looked up once per device (hipGetSymbolAddress) on the first call with that device
 * current.  The array covers every grid lbm_check_params accepts (LBM_ERR_UNSUPPORTED
 * otherwise).  Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other threads) race and must be ordered by the caller.  Nothing in the
 * array needs clearing: each call writes every partial it reads. */
lbm_status lbm_diagnostics_noalloc(const lbm_params *p, const lbm_state *s, double r_n, double *out,
                                   void *stream);

/* ------------------------------------------------------------------ adjoint */

typedef struct {
    void *adj[2];              /* device: two adjoint population buffers, lbm_adj_bytes() each */
    int32_t cur;               /* buffer holding lambda^{m+1} = dL/df^{m+1} before a step */
    double *g_mu, *g_lam;      /* device, 1 plane each: accumulated dL/dmu, dL/dlam, or NULL */
    double *g_body;            /* device, 2 planes: accumulated dL/db, or NULL.  The three
                                  must be ordinary device memory (not host memory mapped into
                                  the device): lbm_adjoint_step_multi adds to them with FP64
                                  atomic adds, which such memory may not perform */
    const int32_t *probe;      /* device: nprobe node indices (b*nx + a), each in
                                  [0, nx*ny); a cell may repeat (its sources add up).  The
                                  library cannot read device memory before launching: the
                                  kernels skip an index outside the grid and set
                                  LBM_FAULT_PROBE, so callers validate indices on the host */
    const double *ubar;        /* device: 2*nprobe values (component-major), dL/du^N at the probes */
    int32_t nprobe;
    int64_t nsteps;            /* N, the level at which u^N enters the loss */
    void *aux;                 /* device, lbm_aux_bytes(): traction-wall adjoint staging */
    void *gsum;                /* device, lbm_adj_sum_bytes(), zero-filled by the caller before
                                  m = N - 1; F32/F16 storage only (FP64 storage adds to the
                                  gradients directly), required there when any gradient
                                  pointer is set.  The bulk parts of dL/dmu, dL/dlam, dL/db are
                                  summed here in FP32 (4 tiled planes) and moved into the FP64
                                  gradients at every level m with m % 16 == 0, which includes
                                  the last step m = 0; it is zero again after that step */
    /* device, optional: the probe table of these probes (lbm_adjoint_probe_table).  With
     * both set, lbm_adjoint_step adds the probe sources inside its bulk kernel; with either
     * NULL one thread walks the probes after it (its cost grows with nprobe). */
    const uint64_t *probe_mask;
    const double *probe_field;
} lbm_adj_state;

/* Bytes of one adjoint population buffer (24 tiled planes of the compute type). */
size_t lbm_adj_bytes(const lbm_params *p);
/* Bytes of the FP32 gradient block sums (lbm_adj_state.gsum). */
size_t lbm_adj_sum_bytes(const lbm_params *p);

/* One step of the hand-written adjoint of lbm_step, level m (reverse of eq:collision
 * and eq:streaming with the Jacobian actions eq:jacobian-actions and eq:feq-derivative):
 * from lambda^{m+1} in a->adj[a->cur] (zero-filled by the caller before m = N) and the
 * record of U^m, it forms lambda*^m by pull (wall links: transposed rules of
 * eq:boundary-general, traction links also through the boundary Newton solve by the
 * implicit function theorem), dL/dU^m = omega sum_q (f^eq_q)'^T lambda*^m_q + probe and
 * wall sources, lambda^m = (1 - omega) lambda*^m + dL/dU^m into a->adj[1 - a->cur], and
 * adds this level's parts of dL/dmu, dL/dlam, dL/db (bulk parts through a->gsum, see
 * there; the steps must run m = N-1, ..., 0 for the block sums to be folded).  Flips
 * a->cur.
 *   fwd: the forward state (parameters mu, lam, body; pop/ustar are not read).
 *   r_m: body factor at level m.  at_half: boundary data at t^{m+1/2} (step m -> m+1).
 *   record_m: device, U^m as written by lbm_step(record) or lbm_record_state. */
lbm_status lbm_adjoint_step(const lbm_params *p, const lbm_state *fwd, lbm_adj_state *a,
                            int64_t m, double r_m, const lbm_edge_data *at_half,
                            const void *record_m, void *stream);

/* Bytes of the probe mask of lbm_adjoint_step2: one 64-bit word per row of each 64-node
 * tile (bit a mod 64 of word b * T + a / 64 marks node (a, b)). */
size_t lbm_probe_mask_bytes(const lbm_params *p);

/* Fills the probe table that lbm_adjoint_step2 (and lbm_adjoint_step, through
 * a->probe_mask / a->probe_field) reads, from a->probe and a->ubar: mask (device,
 * lbm_probe_mask_bytes()) and field (device, 2 double planes of dL/du^N summed over the
 * probes of each cell, zero away from the probes).  Clears both first (fill kernels, no
 * memset).  Call once per backward pass, after a->probe and a->ubar are set. */
lbm_status lbm_adjoint_probe_table(const lbm_params *p, const lbm_adj_state *a, uint64_t *mask,
                                   double *field, void *stream);

/* Two adjoint levels m and m - 1 in one pass over the grid (temporal blocking of
 * lbm_adjoint_step; lambda^m stays on chip): lambda^{m+1} in a->adj[a->cur] -> lambda^{m-1}
 * in a->adj[1 - a->cur], with the gradient updates and probe sources of both levels.  The
 * result, the block sums and the FP64 gradients are those of lbm_adjoint_step(m) followed
 * by lbm_adjoint_step(m - 1) with the same probe table set in a, bit for bit.  Flips a->cur.
 *   r_m, r_mm1: body factors at levels m and m - 1.
 *   at_half, at_half_prev: boundary data at t^{m+1/2} and t^{m-1/2} (the steps m -> m+1 and
 *     m-1 -> m); may be NULL only when all edges are periodic (LBM_ERR_ARG otherwise).
 *   record_m, record_mm1: device, U^m and U^{m-1} as lbm_adjoint_step reads them.
 *   mask, field: the probe table (lbm_adjoint_probe_table); may be NULL when a->nprobe = 0.
 * On a grid with walls a->aux (lbm_aux_bytes()) is required: the bulk pass leaves lambda^m
 * of the wall lines and first interior lines there, a small kernel completes the wall nodes
 * over both levels, and the traction stages of level m - 1 read lambda^m from those lines.
 * Requires 1 <= m < a->nsteps: level N carries the half-weight probe term and takes
 * lbm_adjoint_step. */
lbm_status lbm_adjoint_step2(const lbm_params *p, const lbm_state *fwd, lbm_adj_state *a,
                             int64_t m, double r_m, double r_mm1, const lbm_edge_data *at_half,
                             const lbm_edge_data *at_half_prev, const void *record_m,
                             const void *record_mm1, const uint64_t *mask, const double *field,
                             void *stream);

/* `levels` adjoint levels (2 to 4), m, m - 1, ..., m - levels + 1, in one pass over a
 * periodic grid (temporal blocking of lbm_adjoint_step; the levels in between stay in
 * registers): lambda^{m+1} in a->adj[a->cur] -> lambda^{m-levels+1} in a->adj[1 - a->cur],
 * with the gradient updates (block sums, their folds into the FP64 gradients) and probe
 * sources of every level.  The result, the block sums and the FP64 gradients are those of
 * lbm_adjoint_step(m), ..., lbm_adjoint_step(m - levels + 1) with the same probe table set
 * in a, bit for bit on every node; the padding nodes of the tiled arrays receive
 * unspecified values.  Flips a->cur.
 *   r: host array of `levels` body factors r(m), r(m - 1), ...
 *   records: host array of `levels` device pointers, U^m, U^{m-1}, ... as lbm_adjoint_step
 *     reads them.
 *   mask, field: the probe table (lbm_adjoint_probe_table); may be NULL when a->nprobe = 0.
 * Requires levels - 1 <= m < a->nsteps (level N carries the half-weight probe term and
 * takes lbm_adjoint_step); LBM_ERR_ARG otherwise.  FP32 and FP16 storage on periodic grids;
 * LBM_ERR_UNSUPPORTED for FP64 storage or a grid with a wall (lbm_adjoint_step2 takes those). */
lbm_status lbm_adjoint_step_multi(const lbm_params *p, const lbm_state *fwd, lbm_adj_state *a,
                                  int64_t m, int levels, const double *r, const void *const *records,
                                  const uint64_t *mask, const double *field, void *stream);

/* Adjoint of lbm_init: from lambda^0 = dL/df(0) in a->adj[a->cur], writes dL/dv0 into
 * g_v0 (device, 2 double planes; includes the direct term of u*^0 = u0 - (dt/2) v0) and
 * adds the initialisation parts of dL/dmu, dL/dlam, dL/db.  v0, u0, Fbar, r0 as given to
 * lbm_init.  Uses a->adj[1 - a->cur] as scratch. */
lbm_status lbm_adjoint_init(const lbm_params *p, const lbm_state *fwd, lbm_adj_state *a,
                            const double *v0, const double *u0, const double *Fbar, double r0,
                            double *g_v0, void *stream);

/* Writes U^n of the current level in record format (6 tiled planes of the compute type). */
lbm_status lbm_record_state(const lbm_params *p, const lbm_state *s, double r_n, void *record,
                            void *stream);

/* ------------------------------------------------------------------ misc */

const char *lbm_status_string(lbm_status st);
/* Library version string. */
const char *lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
