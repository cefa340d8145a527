/*
 * qslater.h -- C ABI of the MI355X (gfx950) Slater-matrix builder.
 *
 * The library computes, for a batch of QMC walkers, the quantities of
 * Scemama, Caffarel, Oseret, Jalby, "Quantum Monte Carlo for large chemical
 * systems" (arXiv:1209.6630):
 *
 *   AOs      chi(r) = (x-Qx)^nx (y-Qy)^ny (z-Qz)^nz sum_k c_k exp(-gamma_k |r-Q|^2)
 *            (section "The quantum Monte Carlo method", critical CPU part,
 *            equations for chi and g), screened as in section "Exploiting the
 *            highly localized character of atomic basis functions";
 *   MOs      phi_i(r) = sum_j a_ij chi_j(r)                    (equation (mo));
 *   products C_n = A B_n, n = 1..5: values, d/dx, d/dy, d/dz, Laplacian
 *            of the MOs at every electron of a spin                (equation (abc));
 *   Slater   D_ij = phi_i(r_j); log|det D|, sign, D^-1 (Slater determinant
 *            equation; inversion step of section "Overall performance");
 *   drift    sum_j D^(1)_{l,ij} D^-1_ji and Laplacian sum_j D^(2)_{l,ij} D^-1_ji
 *            (the two "vector products" equations of the critical CPU part);
 *   adjoint  d(sum_w g_w . logdet_w)/dA and /dR (not in the paper: chain rule
 *            through equation (mo) and the Slater matrix definition).
 *
 * Conventions used by every call:
 *   - AO order: atom-major, shells in the order given, Cartesian components
 *     x,y,z for p and xx,xy,xz,yy,yz,zz for d.  qsl_ao_info reports it.
 *   - Screening: primitive k is kept iff gamma_k * r^2 <= screen_T, decided in
 *     FP64 as r^2 = (dx*dx + dy*dy) + dz*dz without fused multiply-add, in
 *     every precision mode.  A shell with no kept primitive contributes 0.
 *   - Every Cartesian AO has unit norm (the library normalises the raw
 *     contraction weights).
 *   - Electrons of a walker: the first n_up are spin up, the next n_dn down.
 *   - Per spin s with n = n_s: C^s is stored [W][5][n][n] as C[w][c][e][i]
 *     (electron e, MO i fastest); D[i][e] = C[w][0][e][i]; Dinv^s is stored
 *     [W][n][n] as Dinv[w][e][i] with sum_i Dinv[e][i] D[i][e'] = delta.
 *   - Pointers named "device" must be device memory of the current HIP
 *     device; the library never frees caller memory.
 *   - Every call returns a qsl_status; no C++ exception crosses the ABI.
 *     qsl_last_error() returns a thread-local description of the last
 *     failure.  Numerical conditions (singular D, near-tie screening, non
 *     finite values) are reported per walker in `status`, not as errors.
 *   - Calls that take a stream only enqueue work on that stream (a
 *     hipStream_t passed as void*; NULL is the default stream).
 *   - A qsl_system must not be modified (qsl_set_mo) while a call that
 *     reads it is in flight.  Calls on different streams with separate
 *     workspaces may overlap.
 */
#ifndef QSLATER_H
#define QSLATER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QSL_OK = 0,
    QSL_ERR_INVALID_ARG = 1,  /* NULL where required, bad value, bad spin */
    QSL_ERR_UNSUPPORTED = 2,  /* l > 2, too many primitives, size limit   */
    QSL_ERR_SHAPE = 3,        /* sizes that do not match the system       */
    QSL_ERR_WORKSPACE = 4,    /* workspace NULL or smaller than required  */
    QSL_ERR_HIP = 5,          /* a HIP runtime call failed (see last_error) */
    QSL_ERR_OOM = 6           /* device allocation failed                 */
} qsl_status;

/* Arithmetic of the AO->MO products (equation (abc)).  Screening is FP64
 * in every mode; LU, log|det|, inverse, drift and Laplacian are FP64. */
typedef enum {
    QSL_FP64 = 0,   /* AOs FP64, products FP64 (MFMA f64); C is double  */
    QSL_FP32 = 1,   /* AOs FP32, products FP32 (MFMA f32); C is float   */
    QSL_BF16X3 = 2  /* AOs FP32, products as hi/lo BF16 split, three BF16
                       MFMA products with FP32 accumulation; C is float  */
} qsl_mode;

/* Per-walker status bits. */
#define QSL_STATUS_SINGULAR 1u   /* an exact zero pivot: logdet=-inf, sign=0 */
#define QSL_STATUS_NEAR_TIE 2u   /* some kept/dropped primitive had
                                    |gamma r^2 - T| <= 1e-12 T (best effort) */
#define QSL_STATUS_NONFINITE 4u  /* a non-finite logdet/drift/Laplacian     */

/* Limits. */
#define QSL_LMAX 2
#define QSL_PMAX 8               /* primitives per shell */

typedef struct qsl_system qsl_system;

/* System description (host memory; copied by qsl_system_create). */
typedef struct {
    int32_t n_atoms;
    const double* atom_xyz;     /* [n_atoms][3], bohr                           */
    int32_t n_shells;
    const int32_t* shell_atom;  /* [n_shells], non-decreasing (atom-major)      */
    const int32_t* shell_l;     /* [n_shells], 0..QSL_LMAX                      */
    const int32_t* shell_nprim; /* [n_shells], 1..QSL_PMAX                      */
    const double* prim_exp;     /* [sum nprim], gamma_k > 0                      */
    const double* prim_coef;    /* [sum nprim], raw contraction weights d_k      */
    int32_t n_up, n_dn;         /* electrons per spin, n_up >= n_dn >= 0         */
    double screen_T;            /* screening threshold T (<= 0 means 30)        */
    uint32_t flags;             /* reserved, must be 0                           */
} qsl_system_desc;

/*
 * Create a system: validates the description, normalises the contraction
 * weights, builds the AO order and the device tables (atoms, shells,
 * primitives, padded AO slots).  Everything is copied; the caller keeps its
 * arrays.  Allocates device memory on the current device.
 * Errors: INVALID_ARG (NULL, n_up < n_dn, non-finite coordinate, gamma <= 0,
 * shell_atom not non-decreasing or out of range), UNSUPPORTED (l > 2,
 * nprim > QSL_PMAX), OOM, HIP.
 */
qsl_status qsl_system_create(const qsl_system_desc* desc, qsl_system** out);

/* Free a system and its device tables.  NULL is accepted. */
qsl_status qsl_system_destroy(qsl_system* sys);

/* Number of AOs N_b (the column count of A^s). Returns -1 for NULL. */
int64_t qsl_n_basis(const qsl_system* sys);

/*
 * AO order: for AO j, ao_atom[j], ao_shell[j] and its powers
 * ao_nxyz[3j..3j+2] = (nx, ny, nz).  Host arrays of N_b (3 N_b) entries;
 * any may be NULL.
 */
qsl_status qsl_ao_info(const qsl_system* sys, int32_t* ao_atom, int32_t* ao_shell,
                       int8_t* ao_nxyz);

/*
 * Set the MO coefficients a_ij of spin s (0 = up, 1 = down): A is n_s x N_b,
 * row-major with leading dimension ld >= N_b (equation (mo)), in host memory
 * (on_device = 0) or device memory (on_device = 1).  The library keeps its
 * own FP64, FP32 and hi/lo BF16 copies in its padded layout (A is constant
 * between calls).  Enqueued on `stream`; A may be reused once the stream has
 * passed this call (host A: as soon as the call returns).
 * Errors: INVALID_ARG (spin, NULL, ld < N_b), HIP.
 */
qsl_status qsl_set_mo(qsl_system* sys, int32_t spin, const double* A, int64_t ld,
                      int32_t on_device, void* stream);

/* Forward arguments.  Output pointers are device memory.  C and Dinv are
 * required (the inversion reads C_1, the drift reads Dinv); logdet, sign,
 * drift, lap and status may be NULL to skip them. */
typedef struct {
    int64_t W;                /* walkers                                        */
    const double* R;          /* [W][n_up+n_dn][3] device, bohr                  */
    int32_t mode;             /* qsl_mode                                        */
    void* C[2];               /* per spin [W][5][n_s][n_s]: double (FP64) or float */
    double* logdet;           /* [W][2]  natural log |det D^s|                   */
    int8_t* sign;             /* [W][2]  -1, 0, +1                                */
    double* Dinv[2];          /* per spin [W][n_s][n_s]                           */
    double* drift;            /* [W][n_up+n_dn][3]: (1/Det) dDet/dx_e             */
    double* lap;              /* [W][n_up+n_dn]:    (1/Det) lap_e Det             */
    uint32_t* status;         /* [W] QSL_STATUS_* bits                            */
    void* ws;                 /* device workspace (see qsl_workspace_size)        */
    size_t ws_bytes;
} qsl_fwd_args;

/* Workspace selectors of qsl_workspace_size. */
#define QSL_WS_FORWARD 1   /* what qsl_forward needs                       */
#define QSL_WS_BACKWARD 2  /* what qsl_backward needs (covers the forward) */
#define QSL_WS_BOTH 3

/*
 * Device workspace bytes needed by qsl_forward (what = QSL_WS_FORWARD) or
 * qsl_backward (QSL_WS_BACKWARD or QSL_WS_BOTH) for W walkers in `mode`.
 * The forward's regions come first, so a backward-sized workspace serves
 * both calls (not concurrently); a forward-only caller needs less (no
 * walker-group lists, dA accumulator or split G).
 * Errors: INVALID_ARG (NULL, W < 0, bad mode or selector).
 */
qsl_status qsl_workspace_size(const qsl_system* sys, int64_t W, int32_t mode, int32_t what, size_t* bytes);

/*
 * Forward: screening and compaction of the surviving AO windows per tile of
 * electrons, fused AO evaluation + AO->MO products on MFMA, FP64
 * Gauss-Jordan elimination with partial pivoting for log|det|, sign and
 * D^-1, then drift and Laplacian.  Enqueued on `stream`.
 * Errors: INVALID_ARG (NULL R, W < 0, bad mode, MOs of a spin never set),
 * WORKSPACE, UNSUPPORTED (a spin with more electrons than the inversion
 * supports), HIP.
 */
qsl_status qsl_forward(qsl_system* sys, const qsl_fwd_args* args, void* stream);

/*
 * For callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid hipMalloc): the
 * forward of qsl_forward with its workspace taken from a static device array
 * of QSL_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs
 * on until the process ends; args->ws and args->ws_bytes are ignored.  Calls
 * no hipMalloc, hipFree or other allocating routine, and is not timed by
 * qsl_profile_enable.  Every call on one GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other threads) race; nothing
 * in the array needs to start at zero (each call writes what it reads).
 * Outputs equal those of qsl_forward bit for bit.
 * Errors: those of qsl_forward; WORKSPACE when the forward of args->W walkers
 * needs more than QSL_NOALLOC_SCRATCH_BYTES (qsl_workspace_size with
 * QSL_WS_FORWARD gives the need: about 43 MB for 4096 walkers of 434
 * electrons); HIP if the array's device address cannot be found.
 */
#define QSL_NOALLOC_SCRATCH_BYTES (64u << 20)
qsl_status qsl_forward_noalloc(qsl_system* sys, const qsl_fwd_args* args, void* stream);

/* Backward arguments (adjoint of L = sum_w sum_s g[w][s] logdet[w][s]). */
typedef struct {
    int64_t W;
    const double* R;          /* [W][N][3] device, as given to the forward        */
    int32_t mode;             /* products in this mode (as the forward)           */
    const double* Dinv[2];    /* per spin [W][n_s][n_s] from the forward          */
    const double* g_logdet;   /* [W][2] device: dL/dlogdet                        */
    double* dR;               /* [W][N][3] device, overwritten (NULL: skip)       */
    double* dA[2];            /* per spin [n_s][N_b] device (NULL: skip)          */
    int32_t accumulate_dA;    /* 1: dA += ..., 0: dA = ...                        */
    void* ws;
    size_t ws_bytes;
    const double* drift;      /* optional [W][N][3] device: the forward's drift on
                                 the same R; then dR = g drift (see below)       */
} qsl_bwd_args;

/*
 * Backward: recomputes the AO values (never stored by the forward) and
 * accumulates dA = sum_w G chi over walkers, G = g D^-1: in FP32 by
 * electron index (per electron and group of up to 1024 walkers, the slots
 * that survive for some walker of the group, the walkers as the products'
 * contraction dimension), in the other modes by ranges of 32 electrons over
 * groups of up to 128 walkers; sums across groups are FP32 (FP64 in FP64
 * mode) atomic adds, then added to dA in FP64.  dR: with drift
 * given, dR[w][e] = g[w][s(e)] drift[w][e] (0 where g = 0), since
 * d log|det D^s| / dr_e = sum_i D^-1[e][i] grad phi_i(r_e) is the drift
 * ("vector products" equations); without it, G A at the recomputed AO
 * gradients.  Derivatives hold the screened survivor sets fixed.  Walkers
 * flagged singular must have g = 0.  Enqueued on `stream`.
 * Errors: INVALID_ARG, WORKSPACE, HIP.
 */
qsl_status qsl_backward(qsl_system* sys, const qsl_bwd_args* args, void* stream);

/* ------------------------------------------------------------------ plans
 *
 * A plan runs the forward and the adjoint of an uneven batch: several
 * systems (different molecules, electron counts and walker counts) in one
 * precision mode.  Every kernel phase (screening, contraction,
 * inversion, drift/Laplacian, adjoint) is one launch whose blocks walk the
 * work list of all (system, spin, electron tile, MO block) items, largest
 * systems first, instead of one launch per system and spin.  Each Monte
 * Carlo step treats every walker independently (subsection "Parallelizing
 * FN-DMC"), so any mix of walkers and systems can share a launch.
 * The adjoint reuses the forward's screening of the same coordinates.
 */
typedef struct qsl_plan qsl_plan;

/* Plan flags. */
#define QSL_PLAN_GRAPH 1u  /* capture the launch sequence into a HIP graph on
                              the first qsl_plan_launch after a bind or a
                              tuning change, and replay it afterwards       */

/* Runtime tuning parameters of a plan (what qsl_autotune searches, except
 * det_dA, which the caller chooses). */
typedef struct {
    int32_t batched;    /* 1: one launch per phase over the work list of all
                           systems; 0: one launch per system and spin       */
    int32_t adj_group;  /* walkers per dA group of the adjoint, 1..4096;
                           0: min(W, 1024) for the FP32 dA by electron,
                           min(W, 128) for the dA by 32-electron range     */
    int32_t gj_bias;    /* 0: the smallest Gauss-Jordan block shape holding
                           n; 1: the next larger one (when there is one)      */
    int32_t contract_tile; /* FP32 products: 0 = 256 MOs per workgroup, two
                              workgroups per CU; 1 = 128 MOs, three per CU;
                              2 = as 0, each FP32 operand split exactly into
                              three bf16 and the six leading products taken
                              on bf16 MFMA with FP32 accumulation (per
                              product 2^-23 relative against FP32's 2^-24) */
    int32_t persistent; /* 1 (with batched): the products run as resident
                           workgroups taking work items from a device counter
                           (largest systems first) instead of one workgroup
                           per item                                          */
    int32_t det_dA;     /* 1: dA summed without atomics: one adjoint dA
                           launch per 32-electron range, each walker group
                           adding into partial sums of its own (ranges in
                           ascending order), then the partials summed in
                           FP64 in ascending group order: the same dA on
                           every launch, for ceil(W / group) x n x N_b more
                           words of plan workspace per spin; 0: atomic
                           accumulation                                     */
} qsl_tuning;

/*
 * Create a plan over n_sys systems with W[i] walkers each, all in `mode`.
 * flags: QSL_PLAN_GRAPH or 0.  The plan owns its workspace (allocated on the
 * current device at the first launch).  The systems must outlive the plan;
 * their MO coefficients are read at launch time.
 * Errors: INVALID_ARG (n_sys < 1, NULL, W < 0, bad mode or flags), OOM.
 */
qsl_status qsl_plan_create(int32_t n_sys, qsl_system* const* sys, const int64_t* W, int32_t mode,
                           uint32_t flags, qsl_plan** out);

/*
 * Bind the device buffers of system i: `fwd` as for qsl_forward (required;
 * its W and mode must match the plan, ws/ws_bytes are ignored), `bwd` as for
 * qsl_backward, or NULL for a forward-only system (its W and mode must
 * match, bwd->R must equal fwd->R, ws/ws_bytes ignored; with bwd->drift
 * NULL the forward's drift, if bound, serves for dR).  Pointers must
 * stay valid and fixed while the plan is launched (a graph replays them);
 * binding again invalidates a captured graph.  Nothing is enqueued.
 * Errors: INVALID_ARG, SHAPE (W or mode differ from the plan),
 * UNSUPPORTED (a spin with more electrons than the inversion supports).
 */
qsl_status qsl_plan_bind(qsl_plan* plan, int32_t i, const qsl_fwd_args* fwd, const qsl_bwd_args* bwd);

/*
 * Set / read the tuning.  Setting invalidates a captured graph.
 * Errors: INVALID_ARG (NULL, a value out of range).
 */
qsl_status qsl_plan_set_tuning(qsl_plan* plan, const qsl_tuning* t);
qsl_status qsl_plan_get_tuning(const qsl_plan* plan, qsl_tuning* t);

/*
 * Enqueue the forward of every system, then the adjoint of every system
 * bound with `bwd`, on `stream`.  Results equal those of qsl_forward /
 * qsl_backward per system with the same tuning (bit for bit, except dA,
 * whose atomic sums over walker groups may round in any order; with
 * det_dA = 1, dA too is the same on every launch).  The first
 * launch after a bind or a tuning change synchronises `stream`, uploads the
 * work lists and (QSL_PLAN_GRAPH) captures the graph; later launches only
 * enqueue.  Launches of one plan must not overlap.
 * Errors: INVALID_ARG (a system never bound), OOM, HIP.
 */
qsl_status qsl_plan_launch(qsl_plan* plan, void* stream);

/* Free a plan, its workspace and graph.  NULL is accepted. */
qsl_status qsl_plan_destroy(qsl_plan* plan);

/*
 * Autotune: time every candidate tuning (batched 0/1 x adj_group in
 * {0, 16, 32, ..., 1024} x gj_bias 0/1, then, from the fastest of those,
 * the FP32 contraction tile and the persistent launch; det_dA stays as
 * set) on the bound buffers, keep the
 * fastest whose outputs pass a parity self-check against the default
 * tuning (logdet, sign, D^-1, drift, Laplacian and dR of the first and last
 * walkers of every system within 1e-9 relative, dA within 1e-10 (FP64) or
 * 1e-4 (other modes) of its largest entry), and set it on the plan.  With
 * cache_path, a JSON file keyed by device, mode and the shapes of the
 * batch: a hit sets the cached tuning without running anything; a miss
 * tunes and writes the entry.  Overwrites the bound outputs, dA included:
 * while tuning, every run writes dA as if accumulate_dA were 0 (the
 * caller's flags apply again to later launches), so an accumulated dA must
 * be saved by the caller first.  Synchronises `stream`.  `chosen` (may be
 * NULL) receives the tuning; on failure the previous tuning stays set.
 * Errors: INVALID_ARG, HIP, OOM; UNSUPPORTED if no candidate passes.
 */
qsl_status qsl_autotune(qsl_plan* plan, const char* cache_path, void* stream, qsl_tuning* chosen);

/* ------------------------------------------------------- determinants
 *
 * Psi_det = sum_K c_K Det_K_up Det_K_dn (the trial wavefunction equation of
 * section "The quantum Monte Carlo method"): every determinant takes n_s of
 * the n_orb >= n_s orbitals of an orbital set per spin.
 */

/*
 * Orbital set of spin s: A is n_orb x N_b (n_orb >= the spin's electrons),
 * row-major with leading dimension ld, host (on_device = 0) or device memory.
 * It replaces the MO coefficients of that spin; qsl_forward, qsl_backward
 * and plans need n_orb equal to the spin's electrons again (qsl_set_mo) and
 * report SHAPE otherwise.  May reallocate the library's MO copies (it then
 * synchronises `stream`; plans of the system rebuild their work lists at
 * their next launch).  Errors: INVALID_ARG, OOM, HIP.
 */
qsl_status qsl_set_orbitals(qsl_system* sys, int32_t spin, const double* A, int32_t n_orb, int64_t ld,
                            int32_t on_device, void* stream);

typedef struct {
    int64_t W;
    const double* R;          /* [W][N][3] device                                      */
    int32_t mode;             /* qsl_mode of the products                               */
    int32_t n_det;            /* >= 1                                                   */
    const int32_t* occ;       /* host [n_det][n_up + n_dn]: orbital indices of each
                                 determinant, its n_up spin-up orbitals then its n_dn
                                 spin-down ones (rows of the spin's orbital set)      */
    const double* coef;       /* host [n_det]: c_K                                      */
    double* logpsi;           /* [W] log|Psi_det| (-inf where it vanishes)              */
    int8_t* sign;             /* [W] sign of Psi_det                                    */
    double* drift;            /* [W][N][3] grad Psi_det / Psi_det (may be NULL)         */
    double* lap;              /* [W][N]    lap_e Psi_det / Psi_det (may be NULL)        */
    uint32_t* status;         /* [W] QSL_STATUS_* bits (may be NULL)                    */
    double* det_logdet;       /* [n_det][W][2] per determinant and spin (may be NULL)  */
    int8_t* det_sign;         /* [n_det][W][2] (may be NULL)                            */
    void* ws;                 /* device workspace of qsl_multidet_workspace_size        */
    size_t ws_bytes;
} qsl_multidet_args;

qsl_status qsl_multidet_workspace_size(const qsl_system* sys, int64_t W, int32_t mode, int32_t n_det, size_t* bytes);

/*
 * The products of the whole orbital set once per spin (equation (abc)),
 * then for each determinant: its columns of C gathered, the FP64
 * Gauss-Jordan log|det|, sign and inverse, its drift and Laplacian ratio;
 * then per walker the max-shifted combination
 *   log|Psi_det| = m + log|S|, S = sum_K sign_K e^(log|c_K Det_K| - m),
 *   drift_e = sum_K w_K drift_K(e), lap_e = sum_K w_K lap_K(e),
 *   w_K = c_K Det_K_up Det_K_dn / Psi_det.
 * Uploads occ and coef with asynchronous copies from host memory (not for
 * graph capture).  Errors: INVALID_ARG (NULL, orbital index out of range,
 * non-finite c_K, orbitals never set), UNSUPPORTED, WORKSPACE, HIP.
 */
qsl_status qsl_multidet_forward(qsl_system* sys, const qsl_multidet_args* args, void* stream);

/* ------------------------------------------------------------- QMC step
 *
 * One fixed-node diffusion Monte Carlo step around the Slater part (section
 * "The quantum Monte Carlo method"), for Psi = e^J Det_up Det_dn with the
 * Jastrow exponent
 *   J = sum_{i<j} u_ee(r_ij) + sum_{i,alpha} u_en(r_i alpha),
 *   u(r) = a r / (1 + b r),
 *   a = c_ee / 2 (opposite spins), c_ee / 4 (same spin), -c_en Z_alpha (nuclei)
 * (c = 1: the electron-electron and electron-nucleus cusp conditions; the
 * paper leaves the U functions open), the Coulomb Hamiltonian of the
 * electrons and the nuclei of charges Z, and the population reconfigured at
 * a constant number of walkers.  Everything here is FP64.
 */

/*
 * Nuclear charges Z[n_atoms] (host, >= 0) and the Jastrow parameters of a
 * system (b >= 0; c = 0 switches a term off).  Copies Z to the device.
 * Errors: INVALID_ARG, OOM, HIP.
 */
qsl_status qsl_set_jastrow(qsl_system* sys, const double* Z, double c_ee, double b_ee, double c_en, double b_en);

/* Local energy arguments (device pointers). */
typedef struct {
    int64_t W;
    const double* R;          /* [W][N][3] positions                                */
    const double* drift_det;  /* [W][N][3] the forward's drift at R (grad Det / Det) */
    const double* lap_det;    /* [W][N]    the forward's Laplacian ratio at R        */
    const double* logdet;     /* [W][2], and sign [W][2]: the forward's at R         */
    const int8_t* sign;
    double* EL;               /* [W] out: local energy H Psi / Psi                   */
    double* drift;            /* [W][N][3] out: grad Psi / Psi = grad J + drift_det  */
    double* logpsi;           /* [W] out or NULL: J + log|Det_up| + log|Det_dn|      */
    int8_t* psisign;          /* [W] out or NULL: sign of Psi                        */
    double* J;                /* [W] out or NULL: the Jastrow exponent               */
    double* V;                /* [W] out or NULL: the Coulomb potential              */
} qsl_local_args;

/*
 * Local energy (equation (localenergy)) and drift (equation (drift)) of
 * Psi = e^J Det_up Det_dn from the forward's determinant drift and Laplacian
 * ratio: lap_i Psi / Psi = lap_i J + |grad_i J|^2 + 2 grad_i J . drift_det_i
 * + lap_det_i; E_L = -1/2 sum_i lap_i Psi / Psi + V.  One workgroup per
 * walker.  Errors: INVALID_ARG (NULL, jastrow never set), UNSUPPORTED (more
 * than 2048 electrons), HIP.
 */
qsl_status qsl_local_energy(qsl_system* sys, const qsl_local_args* args, void* stream);

/*
 * Drift-diffusion move (equation (proba)): R_out = (R + tau drift) +
 * sqrt(tau) eta over `count` coordinates, each product and sum rounded on
 * its own; eta are the caller's standard normal deviates.  R_out may not
 * overlap R unless equal to it.  Errors: INVALID_ARG (NULL, tau < 0), HIP.
 */
qsl_status qsl_drift_diffuse(int64_t count, const double* R, const double* drift, const double* eta, double tau,
                             double* R_out, void* stream);

/*
 * Branching weights (equation (w)):
 * w = exp(-tau/2 [(EL_new - E_T) + (EL_old - E_T)]), and w = 0 where the move
 * changed the sign of Psi (a node was crossed, which fixed-node walkers
 * cannot) or Psi vanishes.  Errors: INVALID_ARG, HIP.
 */
qsl_status qsl_branch_weights(int64_t W, const double* EL_new, const double* EL_old, const int8_t* sign_new,
                              const int8_t* sign_old, double E_T, double tau, double* w, void* stream);

/*
 * Reconfiguration at a constant number of walkers (subsection
 * "Parallelizing FN-DMC"): new walker m is idx[m], the first walker whose
 * cumulative weight (summed in walker order into cum[W], a device scratch
 * array) exceeds u[m] (the caller's uniform deviate in [0, 1)) times the
 * total; *wsum (device) receives the total, whose ratio to W is this step's
 * population weight.  A non-positive total keeps the population (idx[m] = m).
 * Weights must be finite and >= 0.  Errors: INVALID_ARG, HIP.
 */
qsl_status qsl_reconfigure(int64_t W, const double* w, const double* u, int64_t* idx, double* wsum, double* cum,
                           void* stream);

/* dst[m] = src[idx[m]] for W records of `width` bytes (device; distinct
 * buffers).  Errors: INVALID_ARG, HIP. */
qsl_status qsl_gather_walkers(int64_t W, int64_t width, const int64_t* idx, const void* src, void* dst, void* stream);

/* State and inputs of a DMC step of system sys_index of a plan. */
typedef struct {
    int32_t sys_index;
    int64_t W;                /* the plan's walkers of that system                  */
    double tau, E_T;          /* time step, reference energy                         */
    double* R;                /* [W][N][3] population (in/out); not the plan's R     */
    double* EL;               /* [W] local energy at R (in/out)                      */
    double* drift;            /* [W][N][3] grad Psi / Psi at R (in/out)              */
    int8_t* psisign;          /* [W] sign of Psi at R (in/out)                       */
    double* logpsi;           /* [W] log|Psi| at R (in/out) or NULL                  */
    const double* eta;        /* [W][N][3] standard normal deviates of the step      */
    const double* u;          /* [W] uniform deviates in [0, 1) of the step          */
    int64_t* idx;             /* [W] out: parent of each new walker                  */
    double* wsum;             /* [1] out: total branching weight of the step         */
    void* ws;                 /* device workspace, qsl_dmc_workspace_size bytes      */
    size_t ws_bytes;
} qsl_dmc_args;

qsl_status qsl_dmc_workspace_size(int64_t W, int32_t n_elec, size_t* bytes);

/*
 * State of the population R: copies R to the plan's bound positions, runs
 * the plan (its forward must be bound with drift, lap, logdet and sign; bind
 * it without an adjoint for DMC) and the local energy, writing EL, drift,
 * psisign (and logpsi).  Errors: INVALID_ARG, SHAPE, UNSUPPORTED, HIP.
 */
qsl_status qsl_dmc_init(qsl_plan* plan, const qsl_dmc_args* args, void* stream);

/*
 * One step: the drift-diffusion move of R into the plan's positions, the
 * plan's Slater build there, the local energy, the branching weights
 * against the state at R, the reconfiguration with u, and the gather of the
 * selected walkers' positions and state back into R, EL, drift, psisign
 * (and logpsi).  Only enqueues work.  Errors: as qsl_dmc_init, WORKSPACE.
 */
qsl_status qsl_dmc_step(qsl_plan* plan, const qsl_dmc_args* args, void* stream);

/*
 * Kernel timing (for benchmarks and profilers).  While enabled, every
 * kernel the library enqueues is bracketed by two HIP events recorded on the
 * stream it is launched on; qsl_profile_read synchronises those events and
 * returns, per kernel name, the number of launches and their summed
 * duration in milliseconds.  `reset` = 1 clears the accumulated records.
 * Process-wide; not thread-safe against concurrent enqueues.
 * Errors: INVALID_ARG (NULL count), HIP.
 */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} qsl_kernel_time;

qsl_status qsl_profile_enable(int32_t on);
qsl_status qsl_profile_read(qsl_kernel_time* out, int32_t capacity, int32_t* count, int32_t reset);

/* Text of a status code (static storage). */
const char* qsl_status_string(qsl_status s);

/* Thread-local description of the last error ("" if none). */
const char* qsl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QSLATER_H */
