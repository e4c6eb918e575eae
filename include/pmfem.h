/*
 * pmfem.h -- C ABI of the MI355X (gfx950) PM-FEM effective-field library.
 *
 * The library evaluates the effective field of the periodic micromagnetic
 * finite element method (Ai, Duan, Lomakin, arXiv 2409.13958) on one GPU:
 *
 *   H_eff = H_ex + H_ms (+ a uniform applied field)               (Eq. heff)
 *
 * on a tetrahedral mesh of a 1D-, 2D- or 3D-periodic unit cell with linear
 * (P1) magnetisation (Eq. M_phi). Periodic images on touching cell faces are
 * merged into their lowest common ancestor (Sec. 2.2), the exchange,
 * charge and gradient operators are periodised (Secs. 3.1, 3.2.1), and the
 * magnetostatic potential is the periodic point-charge superposition
 * (Eq. hms_d2) with the element-exact near correction (Eq. hms_d2b),
 * evaluated by the four-step FFT-based adaptive integral method with a
 * periodic Green's function (Sec. 3.2.2). Protruding cells are folded by
 * Eq. shift_hms. Units are SI throughout.
 *
 * Conventions
 *  - Every entry point returns a pmfem_status (0 = success, < 0 = error);
 *    pmfem_last_error() gives a message for the last failure of a context.
 *  - Host arrays passed in are copied; the caller keeps ownership.
 *  - Device arrays (m_dev, h_dev, ...) belong to the caller; they must hold
 *    N' rows in the library's unknown order (see pmfem_query) and live on
 *    the context's device. Work is enqueued on the context's stream (part
 *    of it on one internal stream of the same device that is forked from
 *    and joined back to the context's stream within each call) and the
 *    call returns without synchronising; device errors surface as
 *    PMFEM_EHIP at the latest on the next call.
 *  - A context is not re-entrant: calls on one context must not overlap.
 *  - All setup (pmfem_build) runs on the host in FP64 and uploads once.
 */
#ifndef PMFEM_H
#define PMFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmfem_ctx pmfem_ctx;

typedef enum {
  PMFEM_OK = 0,
  PMFEM_EINVAL = -1,  /* bad argument or material value                    */
  PMFEM_EMESH = -2,   /* invalid mesh (index out of range, volume <= 0)      */
  PMFEM_EPBC = -3,    /* periodic images inside one tetrahedron (too coarse) */
  PMFEM_EGRID = -4,   /* AIM grid unusable (too short, FFT extent not 2,3,5,7-smooth) */
  PMFEM_ENOMEM = -5,  /* host or device allocation failed                   */
  PMFEM_EHIP = -6,    /* HIP runtime error                                  */
  PMFEM_ESTATE = -7,  /* call out of order (e.g. heff before build)         */
  PMFEM_ECONV = -8    /* an iteration did not reach its tolerance           */
} pmfem_status;

/* Field terms for pmfem_heff. */
#define PMFEM_TERM_EX 1u  /* exchange, Eq. hex / lapl_2                  */
#define PMFEM_TERM_MS 2u  /* magnetostatic, Eqs. hms_d1 - hms_d3          */

/*
 * Create a context on HIP device `hip_device` using stream `hip_stream`
 * (a hipStream_t, or NULL for the default stream). hip_device = -1 makes a
 * host-only context: pmfem_build then assembles the operators without any
 * device work and only the pmfem_export call can read them (used to check
 * the host setup); pmfem_heff and pmfem_llg_step return PMFEM_ESTATE.
 */
int pmfem_create(pmfem_ctx** out, int hip_device, void* hip_stream);

/*
 * Mesh (Sec. 2.2): n_nodes coordinates xyz[n][3] in metres and n_tets
 * tetrahedra tets[t][4] (node indices, any orientation) with a region id per
 * tetrahedron. Image nodes of a touching cell are separate nodes here; they
 * are paired by pmfem_build.
 */
int pmfem_set_mesh(pmfem_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_tets,
                   const int32_t* tets, const int32_t* region);

/* Materials per region: saturation magnetisation Ms[r] > 0 (A/m) and
 * exchange stiffness Aex[r] >= 0 (J/m). */
int pmfem_set_materials(pmfem_ctx* ctx, int32_t n_regions, const double* Ms, const double* Aex);

/*
 * Periodicity (Eq. pm): axis_mask bit0 = x, bit1 = y, bit2 = z; L[3] are
 * the periods in metres (ignored on non-periodic axes). Two nodes form a
 * PBC pair when they coincide modulo the lattice (any combination of
 * periods along the periodic axes, Sec. 2.1) within match_tol * max(L, mesh
 * extent) (match_tol <= 0 selects 1e-9); all images of one point merge into
 * one unknown. A tetrahedron holding two images of one point is EPBC.
 */
int pmfem_set_periodicity(pmfem_ctx* ctx, uint32_t axis_mask, const double L[3],
                          double match_tol);

/*
 * AIM parameters (Sec. 3.2.2): grid[3] points per axis; Lagrange order
 * order_p (1..5) of projection/interpolation; near_boxes = r_b (0..3), the
 * per-axis box radius of the precorrection region; z0_radius_edges = kappa,
 * the radius of the element-exact correction in mean edge lengths;
 * precision selects how the grid charges Q and the grid potential U are
 * stored between the kernels of an evaluation (Sec. 3.2.2 steps 1-3; the
 * paper's own path is single precision at a 1e-3 error level, Sec. 4.5):
 * 0 FP32; 1 BF16 (half the grid bytes, about 8 significant bits); 2 BF16
 * with one refinement step, each grid value stored as the BF16 pair
 * hi = bf16(v), lo = bf16(v - hi) and widened to hi + lo before use (the
 * grid bytes of FP32, about 16 significant bits). All arithmetic, the FFT
 * spectrum, K-hat and every other operator stay FP32; the PGF, the
 * precorrection and element-exact assembly stay FP64 on the host. Other
 * values are EINVAL at pmfem_build. pmfem_grid_convolve always takes and
 * returns FP32 grids. On a periodic axis the
 * grid spacing is L/N and the FFT extent is N; on a non-periodic axis the
 * grid spans the mesh and the FFT extent is 2N. FFT extents must be
 * products of the factors 2, 3, 5 and 7 in [4, 512] (powers of two take the
 * radix-2 passes, the others mixed-radix passes; both with x and y of whole
 * z-planes in LDS where a plane fits); periodic axes need N >= 2 (r_b + p) + 1.
 */
int pmfem_set_aim(pmfem_ctx* ctx, const int32_t grid[3], int32_t order_p, int32_t near_boxes,
                  double z0_radius_edges, int32_t precision);

/*
 * Kernel form of one stage of the evaluation; the results agree within
 * FP32 rounding order. stage "anterp": 1 tile gather, 2 line gather, 3 tile
 * scatter (per-workgroup LDS sums in a fixed order, then a fixed-order sum of
 * the overlapping tile footprints);
 * "interp" (interpolation + precorrection): 1 narrow observer tiles (at
 * most 4 boxes along x), 2 the largest tiles whose staging fits in LDS;
 * "fft": 1 separate x, y, z passes, 2 whole z-planes in LDS for x and y;
 * "spmv" (charges, element correction, exchange and gradient rows): 4, 8
 * or 16 lanes per row on both patterns. variant 0 (the default) picks the
 * scatter anterpolation (3) and the staged forms (2) of the other stages
 * wherever their LDS plans fit, and per pattern the lanes that give each
 * about four entries of a mean row. May be called before or after
 * pmfem_build; EINVAL if the stage or variant is unknown or a forced form
 * does not fit the built problem (the previous choice is kept).
 */
int pmfem_set_variant(pmfem_ctx* ctx, const char* stage, int32_t variant);

/*
 * Build all operators on the host in FP64 (PBC pairs and LCA merge,
 * periodised P1 operators, grid PGF and its spectrum, precorrection and
 * element-exact correction), round them once to FP32 and upload them.
 * Errors: EINVAL, EMESH, EPBC, EGRID, ENOMEM, EHIP, ESTATE (inputs missing).
 */
int pmfem_build(pmfem_ctx* ctx);

/*
 * Sizes and permutations after pmfem_build. n_unknowns = N'.
 * unknown_of_node[N] (or NULL) maps every mesh node to its unknown;
 * node_of_unknown[N'] (or NULL) gives the LCA representative node (the
 * smallest node index of its class). bytes_per_eval (or NULL) receives the
 * algorithmic HBM bytes of one pmfem_heff call with both terms.
 */
int pmfem_query(pmfem_ctx* ctx, int64_t* n_unknowns, int64_t* unknown_of_node,
                int64_t* node_of_unknown, double* bytes_per_eval);

/*
 * Effective field: m_dev[N'][3] unit vectors (FP32, device) -> h_dev[N'][3]
 * in A/m (FP32, device). terms = PMFEM_TERM_EX | PMFEM_TERM_MS. h_applied
 * (host, 3 doubles, A/m) or NULL adds a uniform applied field.
 */
int pmfem_heff(pmfem_ctx* ctx, const float* m_dev, float* h_dev, uint32_t terms,
               const double* h_applied);

/*
 * Same as pmfem_heff with both terms, also writing the intermediate
 * per-unknown results to caller device buffers (each may be NULL):
 * q_dev[N'] nodal charges (A m, Eq. hms_d1), u_dev[N'] corrected potential
 * (A, Eq. hms_d2b), hex_dev[N'][3] exchange field (A/m).
 */
int pmfem_heff_parts(pmfem_ctx* ctx, const float* m_dev, float* h_dev, float* q_dev,
                     float* u_dev, float* hex_dev);

/*
 * Grid convolution alone (step 2 of Sec. 3.2.2): q_grid_dev[Nz][Ny][Nx]
 * real grid charges -> u_grid_dev[Nz][Ny][Nx] = (1/4 pi) K * Q (x fastest).
 */
int pmfem_grid_convolve(pmfem_ctx* ctx, const float* q_grid_dev, float* u_grid_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as pmfem_grid_convolve (the same kernels on the same inputs, so
 * bitwise equal), with the half-spectrum work buffer taken from a
 * library-wide static device array instead of the context's storage. The
 * call allocates nothing. The array holds at most 2^21 complex values
 * (16 MiB): EINVAL if N_z * M_y * (M_x / 2 + 1) exceeds that. Each device
 * has one such array (its address is looked up once per device in
 * pmfem_create) and every call on that device shares it, so calls that
 * overlap on one GPU (several streams, threads or contexts) race; it needs
 * no clearing (the forward passes write all of it before it is read).
 */
int pmfem_grid_convolve_noalloc(pmfem_ctx* ctx, const float* q_grid_dev, float* u_grid_dev);

/*
 * LLG time stepping (Eq. llg, unit-vector Landau-Lifshitz form,
 * gamma0 = 2.21276e5 m/(A s)): n_steps classic RK4 steps of size dt (s)
 * with damping alpha on the FP64 master magnetisation m_dev[N'][3]
 * (device), each stage evaluating H_eff in FP32, the norm restored in FP64
 * after every step. h_applied as in pmfem_heff.
 */
int pmfem_llg_step(pmfem_ctx* ctx, double* m_dev, double dt, double alpha, int32_t n_steps,
                   const double* h_applied);

/*
 * pmfem_llg_step through a HIP graph: the first call (and any call whose
 * m_dev, dt, alpha or h_applied differ from the previous one's, or that
 * finds the surrogate switched on or off, or with the surrogate on,
 * re-created, given parameters or trained since) captures the
 * kernels of one RK4 step, with their fork to the library's second stream
 * and back, into a graph on a stream of the library's own; each call then
 * launches that graph n_steps times on the context's stream. The results are
 * those of pmfem_llg_step, bit for bit; small cells, whose steps are bound by
 * kernel launches, gain most. The graph is kept until pmfem_destroy or the
 * next capture. PMFEM_EHIP if capture, instantiation or a launch fails.
 */
int pmfem_llg_step_graph(pmfem_ctx* ctx, double* m_dev, double dt, double alpha, int32_t n_steps,
                         const double* h_applied);

/*
 * LLG time stepping by the implicit midpoint rule (Sec. 2.2 advances the
 * semi-discrete Eq. llg implicitly, with a Newton iteration whose linear
 * systems a preconditioned Krylov method solves): each of n_steps steps of
 * size dt (s) solves x = m + dt f((m + x)/2), f the right side of Eq. llg
 * (unit-vector Landau-Lifshitz form, damping alpha, gamma0 = 2.21276e5
 * m/(A s)), for the FP64 master magnetisation m_dev[N'][3] (device), with the
 * field terms `terms` (PMFEM_TERM_EX | PMFEM_TERM_MS) plus h_applied (host,
 * 3 doubles, A/m, or NULL). Newton's linear systems are solved by GMRES of
 * at most krylov_dim (<= 60; <= 0 selects 30) vectors, right-preconditioned
 * by the inverse of each node's 3x3 diagonal block of the Jacobian (the field
 * operator replaced by its exchange diagonal); each Krylov vector costs one
 * FP32 field evaluation. A step ends when the root mean square of the
 * residual x - m - dt f((m + x)/2) per component is <= newton_tol (<= 0
 * selects 1e-8; the FP32 field bounds what is reachable, about
 * 1e-7 dt gamma0 |H|). The rule keeps |m| = 1 up to that tolerance without
 * renormalisation. iterations (host, 2 int32, or NULL) receives the Newton and
 * the Krylov iterations of the call. PMFEM_ECONV if a step's Newton iteration
 * does not reach the tolerance in 30 iterations, or stops decreasing for 3
 * (m_dev then holds the last completed step; the message lists the
 * residuals). The first call allocates the solver's device workspace
 * (kept until pmfem_destroy; (krylov_dim + 1) vectors of 24 N' bytes and a
 * few more). Synchronises.
 */
int pmfem_llg_implicit(pmfem_ctx* ctx, double* m_dev, double dt, double alpha, int32_t n_steps,
                       uint32_t terms, const double* h_applied, double newton_tol,
                       int32_t krylov_dim, int32_t* iterations);

/*
 * The midpoint rule of pmfem_llg_implicit with an adaptive time step, as a
 * predictor-corrector pair (the time-step adaptive midpoint scheme of
 * Sec. 2.2 and Sec. 5; its formulas here are this library's choice): it
 * advances m_dev[N'][3] (FP64, device) from t = 0 to t_end (s). The
 * predictor extrapolates the midpoint slopes of the last two accepted
 * steps linearly to the new step's midpoint; Newton (as in
 * pmfem_llg_implicit, from the predictor, tolerance newton_tol, <= 0
 * selects 0.1 lte_tol) corrects it, at least once even where the predictor
 * already meets the tolerance. From the third accepted step on, the
 * local error estimate |C / (C - C_p)| rms(x_c - x_p) per component
 * (Milne's device: C = 1/12 the midpoint rule's constant for a linear right
 * side, C_p the predictor's for the step sizes at hand, history errors
 * included) must be <= lte_tol, else the step is rejected; the next step is
 * h min(2, max(0.2, 0.9 (lte_tol / E)^(1/3))), at most 0.9 h after a
 * rejection. A Newton iteration that fails (10 iterations, 3 without
 * progress, or a residual three times its first) halves the step. Each
 * accepted state is renormalised per node (the rule keeps |m| up to the
 * Newton residual, an rms that a few nodes could exceed). *dt
 * (host) is the first trial step on entry and the proposed next step on
 * return. stats (host, 5 int32, or NULL): accepted steps, steps rejected by
 * the error estimate, steps rejected for a failed Newton iteration, Newton
 * iterations, Krylov iterations. dt_log (host, dt_log_cap doubles,
 * or NULL with cap 0) receives the step size of the first dt_log_cap
 * attempts in order, negated for the rejected ones. max_steps
 * (<= 0 selects 1e6) bounds the accepted steps. PMFEM_ECONV when the step
 * limit is reached or the step falls below 1e-9 t_end (m_dev then holds the
 * last accepted state); PMFEM_EINVAL for bad arguments. Allocates the
 * workspace of pmfem_llg_implicit plus 72 N' bytes on its first call.
 * Synchronises.
 */
int pmfem_llg_implicit_adaptive(pmfem_ctx* ctx, double* m_dev, double t_end, double* dt,
                                double alpha, uint32_t terms, const double* h_applied,
                                double lte_tol, double newton_tol, int32_t krylov_dim,
                                int32_t max_steps, int32_t* stats, double* dt_log,
                                int32_t dt_log_cap);

/*
 * Time-step adaptive BDF2 (the step-adaptive BDF scheme that the paper's
 * timed dynamics run uses, Sec. 2.2 and Sec. 5; its formulas here are this
 * library's choice), with the arguments, Newton-GMRES corrector, step
 * control, renormalisation, statistics and errors of
 * pmfem_llg_implicit_adaptive. The first step is backward Euler,
 * x = m + h f(x); the later ones variable-step BDF2,
 * x = a m - b m_prev + beta h f(x) with w = h / h_prev, a = (1 + w)^2 /
 * (1 + 2 w), b = w^2 / (1 + 2 w), beta = (1 + w) / (1 + 2 w). The predictor
 * extrapolates the line through the last two states or the quadratic
 * through the last three; from the third accepted step on, the local error
 * estimate is h / (h + h1 + h2) times the rms per component of the
 * corrector-predictor gap (h1, h2 the previous steps). BDF2 damps the stiff
 * exchange modes that the midpoint rule carries undamped.
 */
int pmfem_llg_bdf2_adaptive(pmfem_ctx* ctx, double* m_dev, double t_end, double* dt,
                            double alpha, uint32_t terms, const double* h_applied,
                            double lte_tol, double newton_tol, int32_t krylov_dim,
                            int32_t max_steps, int32_t* stats, double* dt_log,
                            int32_t dt_log_cap);

/*
 * Energies in J for the FP64 magnetisation m_dev[N'][3] (device):
 * exchange E_ex = m.K m and magnetostatic E_ms = (mu0/2) q.u. Synchronises.
 */
int pmfem_energy(pmfem_ctx* ctx, const double* m_dev, double* e_ex, double* e_ms);

/*
 * Kernel timing with HIP events on the context's stream. After
 * pmfem_profile_begin(ctx, max_calls), every pmfem_heff call (up to
 * max_calls) records an event pair around each of its kernels;
 * pmfem_profile_end synchronises and returns, for each of the n_kernels
 * (<= 16) kernels in launch order, the summed milliseconds ms[k], the launch
 * count count[k] and its name into names[k] (at most 31 characters + NUL).
 */
int pmfem_profile_begin(pmfem_ctx* ctx, int32_t max_calls);
int pmfem_profile_end(pmfem_ctx* ctx, int32_t* n_kernels, double* ms, int32_t* count,
                      char (*names)[32]);

/*
 * Host copies of an assembled operator, for validation of the setup.
 * name selects the array (see the table in the library source: "mu",
 * "loc_rowptr", "loc_col", "loc_val", "z0_rowptr", "z0_col", "z0_val",
 * "p_rowptr", "p_col", "p_val", "pos", "khat", "kgrid", "box_start",
 * "grid_info"; the scatter anterpolation's tiles: "sc_plan" (int32 tb[3],
 * nt[3], fd[3], fsize), "sc_list" (int32 pairs: unknown, stencil offset in
 * its tile's footprint), "sc_lstart", "sc_tab" (int32 pairs (tile, footprint
 * offset), two per grid index, x then y then z; tile -1 when absent)). With
 * out == NULL only *count (elements) and *elem_bytes are set; otherwise
 * *count elements are copied to out.
 */
int pmfem_export(pmfem_ctx* ctx, const char* name, void* out, int64_t* count,
                 int32_t* elem_bytes);

/*
 * Periodic Green's function of the Laplacian (Eq. 2 at zero Bloch phase,
 * Ewald-regularised; 3D zero cell average, 2D and 1D keeping the
 * -2 pi |z| / A and -(2/L) ln(rho/L) far fields) at n points r[n][3]
 * (metres) into out[n]; a point on a lattice site returns the regular part
 * lim (G - 1/r). Host-only, FP64; eta <= 0 selects the default splitting.
 */
int pmfem_pgf_eval(uint32_t axis_mask, const double L[3], double eta, int64_t n,
                   const double* r, double* out);

/*
 * Autotuner: picks the kernel form of every stage (pmfem_set_variant's
 * stages "anterp", "interp", "fft", "spmv") by coordinate descent, two
 * passes, each candidate timed over `trials` whole evaluations with HIP
 * events (the stages overlap on two streams, so the whole evaluation is the
 * objective). The choice stays set on the context; chosen (host, 4 int32, or
 * NULL) receives it in stage order ("spmv" 0: lanes chosen per pattern from
 * its mean row length), best_ms (or NULL) the mean milliseconds
 * per evaluation of that choice. Synchronises; uses the context's own work
 * buffers as input, so it leaves no caller data changed.
 */
int pmfem_autotune(pmfem_ctx* ctx, int32_t trials, int32_t* chosen, double* best_ms);

/*
 * Batches of independent unit cells (the batched-cell workload: many small
 * periodic cells, each with its own mesh, periods, materials and grid; no
 * data flows between cells). A batch evaluates every cell with one kernel
 * launch per stage for all cells: the exchange, charge, element-correction
 * and gradient operators of the cells concatenated block-diagonally, and the
 * anterpolation, FFT and interpolation kernels in multi-cell form (each
 * workgroup finds its cell in a table). Per cell the arithmetic is that of
 * pmfem_heff with the scatter anterpolation, whole-plane FFT and large
 * interpolation tiles, so the fields agree with the per-cell calls (bitwise
 * when the cells use those forms and the same SpMV lanes).
 *
 * pmfem_batch_create: cells[n_cells] built contexts on one device with the
 * same Lagrange order and near radius, each fitting those kernel forms;
 * hip_stream (or NULL) is the stream the batch's work goes to (part of it on
 * an internal second stream forked from and joined back to it within each
 * call); spmv_lanes 0 picks the SpMV lanes from the mean row lengths, else
 * 4, 8 or 16. The batch copies the cells' local operators; it uses each
 * cell's grid work buffers, so a cell must not be used by other calls while a
 * batch call on it is in flight, and must outlive the batch. Errors: EINVAL
 * (no cells, a repeated cell, different devices, orders or radii, a cell
 * whose plans do not fit), ESTATE (a cell not built), ENOMEM, EHIP; on a
 * set-up error *out still receives the batch (for pmfem_batch_last_error; it
 * must be destroyed), unless it could not be made (then *out is NULL).
 */
typedef struct pmfem_batch pmfem_batch;
int pmfem_batch_create(pmfem_batch** out, int32_t n_cells, pmfem_ctx* const* cells,
                       void* hip_stream, int32_t spmv_lanes);
/* n_unknowns = sum of the cells' N'; cell_offsets[n_cells + 1] (or NULL) the
 * first row of every cell in the packed vectors; bytes_per_eval (or NULL) the
 * sum of the cells' algorithmic bytes per evaluation. */
int pmfem_batch_query(pmfem_batch* b, int64_t* n_unknowns, int64_t* cell_offsets,
                      double* bytes_per_eval);
/* pmfem_heff of every cell: m_dev, h_dev [n_unknowns][3] (device), the cells'
 * unknowns packed in cell order, each cell in its own unknown order. */
int pmfem_batch_heff(pmfem_batch* b, const float* m_dev, float* h_dev, uint32_t terms);
/* n_steps RK4 steps (as pmfem_llg_step, no applied field) of every cell on the
 * packed FP64 master magnetisation m_dev[n_unknowns][3]. */
int pmfem_batch_llg_step(pmfem_batch* b, double* m_dev, double dt, double alpha,
                         int32_t n_steps);
/*
 * pmfem_batch_llg_step through a HIP graph, as pmfem_llg_step_graph for one
 * context: one RK4 step of the whole batch is captured (again when m_dev,
 * dt or alpha change) and launched n_steps times on the batch's stream; the
 * results are those of pmfem_batch_llg_step, bit for bit.
 */
int pmfem_batch_llg_step_graph(pmfem_batch* b, double* m_dev, double dt, double alpha,
                               int32_t n_steps);
const char* pmfem_batch_last_error(const pmfem_batch* b);
void pmfem_batch_destroy(pmfem_batch* b);

/*
 * Learned surrogate of the grid convolution: the second of the four AIM steps
 * (Sec. 3.2.2: the grid charges Q convolved with the periodic Green's
 * function to give the grid potential U, done by FFT in pmfem_heff) replaced
 * by a network of 3x3x3 convolution layers on the same [nz][ny][nx] FP32 grid
 * (x fastest), circular along x and y and zero-padded along z; for films
 * (periodic along x and y only) with the FP32 grid (precision 0). Anterpolation,
 * interpolation, precorrection and the local operators are unchanged.
 *
 * Network: layer 0 maps 1 -> 32 channels, layers 1 .. depth-2 map 32 -> 32,
 * layer depth-1 maps 32 -> 1, ReLU after every layer but the last. Input
 * Q s_in, output times s_out. Parameter vector (FP32), layer by layer:
 * W[co][ci][3][3][3] (index [dz+1][dy+1][dx+1] for the input offset) then
 * b[co]. The kernels use the weights rounded to BF16 (round to nearest even;
 * biases FP32) and accumulate in FP32; the 32 -> 32 layers run on the matrix
 * cores. bf16_activations = 0 keeps FP32 accuracy in those layers by
 * multiplying a BF16 high part and a BF16 remainder of every activation; 1
 * multiplies the BF16-rounded activations only.
 *
 * pmfem_surrogate_init: (re)creates the network of the built context with
 * He-normal weights drawn from seed, zero biases and unset scales. EINVAL for
 * depth outside [2, 12], a cell that is not a film, precision != 0; ENOMEM.
 * The other calls return ESTATE before init; apply, loss_grad, enable(1) and
 * llg_step_judged also while the scales are unset.
 */
int pmfem_surrogate_init(pmfem_ctx* ctx, int32_t depth, uint64_t seed, int32_t bf16_activations);
int pmfem_surrogate_param_count(pmfem_ctx* ctx, int64_t* count);
/* params[count] (host, FP32; count must equal the parameter count) replaces
 * the weights and resets the optimiser; scales[2] = {s_in, s_out} (host,
 * positive) or NULL to keep them. get copies them out (params or scales may
 * be NULL). */
int pmfem_surrogate_set_params(pmfem_ctx* ctx, const float* params, int64_t count,
                               const double* scales);
int pmfem_surrogate_get_params(pmfem_ctx* ctx, float* params, int64_t count, double* scales);
/* u_grid_dev = surrogate(q_grid_dev), device [nz][ny][nx] FP32 buffers of the
 * context's grid (they may be the same buffer); enqueued on the context's
 * stream. */
int pmfem_surrogate_apply(pmfem_ctx* ctx, const float* q_grid_dev, float* u_grid_dev);
/* reps applications (as pmfem_surrogate_apply) with HIP events on the
 * context's stream around every layer: ms_per_layer[depth] (host) the mean
 * milliseconds of each layer's kernel. Synchronous. */
int pmfem_surrogate_profile(pmfem_ctx* ctx, const float* q_grid_dev, float* u_grid_dev,
                            int32_t reps, double* ms_per_layer);
/* One forward and backward pass: y = network(q s_in) (before s_out), loss =
 * mean over the grid points of (y - t)^2 with t_grid_dev in network units,
 * grad[count] (host, or NULL) its gradient with respect to the parameter
 * vector, loss (host, or NULL). Synchronous. */
int pmfem_surrogate_loss_grad(pmfem_ctx* ctx, const float* q_grid_dev, const float* t_grid_dev,
                              double* loss, float* grad, int64_t count);
/* A synthetic magnetisation texture on the unknowns, m_dev[N'][3] FP64
 * (device): kind 0 iid uniform on the sphere, 1 a vortex (random centre,
 * core radius, chirality, polarity), 2 a pair of domain walls along x or y
 * (random position, width, domain and turning directions); parameters drawn
 * from seed. */
int pmfem_surrogate_texture(pmfem_ctx* ctx, int32_t kind, uint64_t seed, double* m_dev);
/* Trains on n_pairs AIM pairs, each a fresh texture (kinds: bit k enables
 * kind k, used in turn) whose grid charges and FFT-convolved potential the
 * plain AIM of this context produces; one Adam step (lr, beta 0.9 / 0.999)
 * per pair on the mean-squared error of the potential in network units. The
 * first pair sets unset scales (unit mean square at input and output).
 * loss_log[n_pairs] (host, or NULL) receives each pair's loss before its
 * step. Synchronous. */
int pmfem_surrogate_train(pmfem_ctx* ctx, int32_t n_pairs, double lr, uint64_t seed,
                          uint32_t kinds, double* loss_log);
/* on != 0: every field evaluation of the context (pmfem_heff, heff_parts,
 * energy, the RK4 and implicit steppers) uses the surrogate in place of the
 * FFT convolution until disabled; pmfem_grid_convolve, pmfem_autotune (which
 * times the plain forms) and batches (pmfem_batch_*) keep the FFT. */
int pmfem_surrogate_enable(pmfem_ctx* ctx, int32_t on);
/*
 * n_steps RK4 steps (as pmfem_llg_step) with the surrogate, judged by the
 * plain AIM: before every check_every-th step (from the first) the
 * magnetostatic field of the current state is evaluated both ways, error =
 * |H_sur - H_aim| / |H_aim| (2-norms over all unknowns; |H_sur - H_aim| if
 * H_aim is zero, as for an in-plane uniform film); once an error
 * exceeds tol the rest of the steps use the FFT convolution. report[4]
 * (host, or NULL): checks made, largest and last error, the step of the
 * fallback (-1 if none). Synchronises at every check.
 */
int pmfem_llg_step_judged(pmfem_ctx* ctx, double* m_dev, double dt, double alpha,
                          int32_t n_steps, const double* h_applied, int32_t check_every,
                          double tol, double* report);

const char* pmfem_last_error(const pmfem_ctx* ctx);

void pmfem_destroy(pmfem_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PMFEM_H */
