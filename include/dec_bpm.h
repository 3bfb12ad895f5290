/*
 * dec_bpm.h - C ABI of the MI355X (gfx950) DEC beam-propagation library.
 *
 * The library marches the nonlinear Schroedinger equation along z on an
 * unstructured triangular mesh of the transverse plane, with the discrete
 * exterior calculus (DEC) operators of the paper:
 *
 *   i dPsi/dz = H_lin Psi - gamma (M |Psi|^2) Psi - i w Psi,
 *   H_lin     = p1 L + beta4 L^2 - diag(v + dn),
 *   L         = H0^{-1} D0^T H1 D0     (Eq. 11, stiffness part; L ~ -Laplacian),
 *   M         = H0^{-1} Q^T D Q         (Eq. 14; or diag(chibar), "lumped"),
 *   v         = H0^{-1} H0(V)           (per-triangle pulse potential, "Discrete Hodge star").
 *
 * Sign reading: Table I gives the Laplacian as -H0^{-1} D0^T H1 D0 and Eq. 1
 * puts -p1 Laplacian on the right-hand side, so the stiffness enters H_lin
 * with a plus sign (Eq. 11 as printed would flip it); the potential guides and
 * the Kerr term focuses.  The higher-order term is the cascaded product of
 * Table I with coefficient +beta4.
 *
 * One z step of length h is the Strang composition
 *   NL(h/2) -> LIN(h) -> NL(h/2),
 * where LIN(h) is one classical fourth-order Runge-Kutta step of
 * dPsi/dz = -i H_lin Psi (the explicit RK4 the paper names for DEC-BPM) and
 * NL(tau) is the exact flow of the Kerr phase and absorber damping:
 *   psi_p <- psi_p e^{-w_p tau} exp(i gamma sum_q M_pq |psi_q|^2 phi(w_q, tau)),
 *   phi(w, tau) = (1 - e^{-2 w tau}) / (2 w).
 * Consecutive half steps of successive z steps are merged into one NL(h).
 *
 * Conventions shared by every call:
 *  - Fields are complex vectors over the vertices in the CALLER's vertex
 *    order: interleaved (re, im) pairs of float (DEC_BPM_C64) or double
 *    (DEC_BPM_C128), contiguous, 8/16-byte aligned, in DEVICE memory owned by
 *    the caller.  The library never frees caller memory and keeps no pointer
 *    to it after a call returns.
 *  - "stream" is a hipStream_t (NULL = the null stream).  Every call is
 *    asynchronous on that stream unless it says it synchronises.
 *  - Return value: DEC_BPM_OK (0) or a negative DEC_BPM_E* code; the message
 *    is available from dec_bpm_last_error() on the same thread.  Arguments
 *    are validated before any device work, so a rejected call changes
 *    nothing.  No C++ exception or abort crosses this interface.
 *  - A handle must not be used from two threads at once; distinct handles are
 *    independent.
 */
#ifndef DEC_BPM_H
#define DEC_BPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dec_bpm_s* dec_bpm_t;
typedef struct dec_bpm_batch_s* dec_bpm_batch_t;

enum {
  DEC_BPM_OK = 0,
  DEC_BPM_EINVAL = -1,     /* bad argument (NULL pointer, size, option)          */
  DEC_BPM_EMESH = -2,      /* degenerate / non-manifold / inconsistent mesh      */
  DEC_BPM_EUNSTABLE = -3,  /* dz * rho(H_lin) exceeds the RK4 stability margin   */
  DEC_BPM_ENOMEM = -4,     /* device or host allocation failed                   */
  DEC_BPM_EHIP = -5,       /* a HIP runtime call failed                          */
  DEC_BPM_ENONFINITE = -6, /* NaN/Inf found in a field                           */
  DEC_BPM_EWORKSPACE = -7, /* workspace too small or not matching the run        */
  DEC_BPM_ENODEVICE = -8   /* handle was created host-only; no device work       */
};

typedef enum { DEC_BPM_C64 = 1, DEC_BPM_C128 = 2 } dec_bpm_dtype;
typedef enum { DEC_BPM_NL_DEC = 0, DEC_BPM_NL_LUMPED = 1 } dec_bpm_nl;
typedef enum { DEC_BPM_N_KERR = 0, DEC_BPM_N_SATURABLE = 1, DEC_BPM_N_CUBIC_QUINTIC = 2 } dec_bpm_response;

typedef struct {
  uint32_t struct_size;   /* sizeof(dec_bpm_options); set by dec_bpm_default_options */
  int32_t dtype;          /* dec_bpm_dtype, default DEC_BPM_C64                       */
  double p1;              /* coefficient of L, default 0.5                           */
  double beta4;           /* coefficient of L^2 (Table I cascaded product), default 0 */
  int32_t nonlinearity;   /* dec_bpm_nl, default DEC_BPM_NL_DEC (Eq. 14)              */
  int32_t reorder;        /* 1: Hilbert space-filling-curve vertex order (default)    */
  const double* chi_tri;  /* [T] Kerr coefficient per triangle (Eq. 14), NULL = 1     */
  int32_t host_only;      /* 1: assemble on the host only (no device allocation);
                             for dec_bpm_export_operators and argument checks        */
  int32_t block_size;     /* threads per workgroup, 0 = library default / autotuned   */
  int32_t steps_per_graph;/* z steps captured per hipGraph, 0 = default; 1 disables   */
  /* Perfectly matched layer in place of (or beside) the absorber, by radial
   * complex stretching of the Hodge stars (the paper's proposal for long
   * distances; the construction is this library's): r~ = r + i S(r),
   * S' = sigma(r) = pml_sigma ((r - pml_r0)/(pml_r1 - pml_r0))^2 for r > pml_r0,
   * centre at the origin.  L becomes H0~^{-1} D0^T H1~ D0 with the dual areas
   * times s_r s_t and the Galerkin H1 with the tensor (s_t/s_r) rr^T +
   * (s_r/s_t) tt^T (s_r = 1 + i sigma, s_t = r~/r, taken at each triangle's
   * centroid); v, M and the power keep the real H0.  pml_sigma = 0: none.
   * Needs 0 < pml_r0 < pml_r1, no beta4 term and rows of at most 12
   * neighbours; the handle then runs dec_bpm_propagate and
   * dec_bpm_propagate_unsplit on the one-kernel step (fused = 2) or, in
   * complex64 when every tile fits at once, the persistent launch (fused = 3),
   * dec_bpm_propagate_adaptive on its trial tiles with complex weights,
   * kerr_step/diagnostics (Hamiltonian NaN), and the checkpointed forward
   * and adjoint on the one-kernel step tiles; the entry points whose kernels
   * apply a real L (apply, linear_step, find_mode, batches) return EINVAL.
   * The stability check uses the unstretched operator's spectral radius,
   * which bounds the stretched one's. */
  double pml_r0, pml_r1, pml_sigma;
  /* Eq. 1 in full: H_lin = p1 L + beta4 L^2 + p3 L^3 + p4 L^4 - diag(v), and
   * the Kerr response N(I) in place of I = |psi|^2 (DEC_BPM_N_KERR, default;
   * DEC_BPM_N_SATURABLE: I / (1 + I / nl_param), nl_param = I_s > 0;
   * DEC_BPM_N_CUBIC_QUINTIC: I - nl_param I^2, nl_param >= 0).  The Kerr
   * substep stays the exact flow: Theta = M (integral over the substep of
   * N(|psi|^2 e^{-2 w z}), in closed form).  A non-Kerr response runs on
   * every split-step launch mode (the tile kernels' Kerr phase takes the
   * flow integral of the response).  p3 or p4 non-zero runs the five-kernel
   * path (fused = 0: the split step's tile kernels cover at most two products
   * per stage); its RK4 stages then run as one tile kernel each, the operator
   * sum by Horner in LDS on tiles of four halo rings (three without p4), or,
   * with DEC_BPM_GEN_TILES=0 in the environment at handle creation, as chains
   * of gather launches.  With either, the
   * checkpointed forward and adjoint, apply(H), batches, unsplit, adaptive
   * and find_mode return EINVAL (their kernels are written for the Kerr
   * right-hand side and terms up to L^2), and diagnostics report a NaN
   * Hamiltonian. */
  double p3, p4;
  int32_t nl_kind;
  double nl_param;
} dec_bpm_options;

/* Fill *opt with the defaults above. */
void dec_bpm_default_options(dec_bpm_options* opt);

/* Thread-local message describing the last failure on this thread. */
const char* dec_bpm_last_error(void);

/* Library version string. */
const char* dec_bpm_version(void);

/*
 * Build the operators of the semi-discrete ODE (Eq. 10) for one mesh.
 *   xy[2*n_vert]        vertex coordinates (x0, y0, x1, y1, ...), host memory
 *   tri[3*n_tri]        vertex indices per triangle, host memory; any
 *                       orientation (each triangle is re-ordered
 *                       counter-clockwise, the paper's convention)
 *   index_tri[n_tri]    potential V_t per triangle, taken at its centroid
 *                       ("Discrete Hodge star"); NULL = 0
 *   absorber_vert[n_vert] absorber strength w_p >= 0 per vertex; NULL = off
 *   opt                 options (NULL = defaults)
 *   out                 receives the handle
 * Host arrays are copied; the caller may free them on return.  Device storage
 * (operators in a space-filling-curve order, work vectors) is owned by the
 * handle until dec_bpm_destroy.  Errors: EINVAL, EMESH (zero-area triangle,
 * index out of range, repeated vertex, edge shared by more than two triangles
 * or traversed twice in one direction, unreferenced vertex), ENOMEM, EHIP.
 */
int dec_bpm_create(const double* xy, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                   const double* index_tri, const double* absorber_vert,
                   const dec_bpm_options* opt, dec_bpm_t* out);

/* Release every resource of the handle (NULL is a no-op). */
void dec_bpm_destroy(dec_bpm_t h);

/* Number of vertices, triangles, edges; nnz of L counting the diagonal. */
int dec_bpm_sizes(dec_bpm_t h, int64_t* n_vert, int64_t* n_tri, int64_t* n_edge, int64_t* nnz);

/* Upper estimate of the spectral radius of H_lin (host Lanczos, FP64); the
 * propagate calls reject dz * rho > 2.5 (the RK4 limit on the imaginary axis
 * is 2 sqrt 2). */
int dec_bpm_spectral_radius(dec_bpm_t h, double* rho);

/*
 * Copy the host-assembled operators out, in the caller's vertex order and FP64
 * (for checks against an independent assembly).  Call once with col/kval/mval
 * NULL to get *nnz, then with arrays of that length.
 *   h0[n], v[n], w[n]   diag of H0, vertex potential (incl. dn), absorber
 *   row_ptr[n+1], col[nnz], kval[nnz]   CSR of K = D0^T H1 D0 (diagonal included)
 *   mval[nnz]           Q^T D Q on the same pattern (NL_DEC) or diag(H0 chibar)
 * Works on host-only handles.
 */
int dec_bpm_export_operators(dec_bpm_t h, double* h0, double* v, double* w, int64_t* nnz,
                             int64_t* row_ptr, int32_t* col, double* kval, double* mval);

/*
 * With a PML (dec_bpm_options.pml_sigma > 0): the complex-stretched operators
 * on the pattern of dec_bpm_export_operators, caller order, interleaved
 * (re, im): h0p[2n] the stretched dual areas, kp[2 nnz] the stretched
 * K~ = D0^T H1~ D0.  Either may be NULL.  EINVAL on a handle without a PML.
 * Works on host-only handles.
 */
int dec_bpm_export_pml(dec_bpm_t h, double* h0p, double* kp);

/*
 * Diagnostics of the vertex order (not in the paper): the tile of the current
 * launch mode that owns each vertex.  The library renumbers the vertices
 * along a Hilbert curve and cuts that order into tiles of *rows_per_tile
 * consecutive rows; tile[i] is the tile of caller vertex i, or -1 (and
 * *rows_per_tile = -1) when the launch mode steps without tiles or the
 * handle is host-only.  tile: host array of n_vert ints, or NULL;
 * rows_per_tile: host int, or NULL.  Errors: EINVAL.
 */
int dec_bpm_vertex_tiles(dec_bpm_t h, int32_t* tile, int32_t* rows_per_tile);

/*
 * Set the per-vertex index perturbation dn: the design variable of the
 * structure optimisation the paper motivates (Abstract, Conclusion); it
 * enters the potential of Eq. 11 as v + dn (added after the triangle-to-vertex
 * averaging of "Discrete Hodge star", unit coupling; derived, the paper gives
 * no coupling).  dn_dev is a device array of n_vert doubles in caller order,
 * or NULL to reset to 0.  Synchronises (dn is also folded into the stability
 * bound on the host, and a digest of its values identifies the operator to
 * the adjoint: installing the same values again restores the same operator).  Errors: EINVAL (misaligned pointer), EUNSTABLE is
 * reported by the next propagate if dn pushes dz rho(H_lin) past the margin.
 */
int dec_bpm_set_index_perturbation(dec_bpm_t h, const double* dn_dev, void* stream);

/* Operator application (parity hooks for the hot kernels), caller order:
 *   DEC_BPM_OP_L:  y = L x          (Eq. 11's stiffness part, Table I Laplacian row);
 *   DEC_BPM_OP_L2: y = L (L x)      (Table I, cascaded higher-order row);
 *   DEC_BPM_OP_H:  y = H_lin x      (the linear part of Eq. 10 with Eq. 11).
 * x and y are distinct device complex vectors of n_vert entries (caller-owned).
 * Errors: EINVAL (bad op, NULL or aliased vectors), ENODEVICE, EHIP. */
enum { DEC_BPM_OP_L = 0, DEC_BPM_OP_L2 = 1, DEC_BPM_OP_H = 2 };
int dec_bpm_apply(dec_bpm_t h, int op, const void* x, void* y, void* stream);

/* One Kerr/absorber substep NL(tau), in place (caller order): the exact flow
 * of the nonlinear term of Eq. 10 with M from Eq. 14 (or the lumped form) and
 * the absorbing imaginary potential (Conclusion: absorbing boundaries); the
 * flow itself is derived (|psi_p| decays as e^{-w tau}, so the phase
 * integrates in closed form).  Errors: EINVAL, ENODEVICE, EHIP. */
int dec_bpm_kerr_step(dec_bpm_t h, void* field, double tau, double gamma, void* stream);

/* One linear RK4 step LIN(h) of dPsi/dz = -i H_lin Psi (Eq. 10 without its
 * nonlinear term; the explicit RK4 of the Introduction), in place, caller
 * order.  Errors: EINVAL, EUNSTABLE, ENODEVICE, EHIP. */
int dec_bpm_linear_step(dec_bpm_t h, void* field, double dz, void* stream);

/*
 * The hot path: n_steps Strang steps of length dz, in place on `field`
 * (caller order).  gamma is the Kerr coefficient (Eq. 1 normalised, q_NL).
 * n_steps == 0 is a no-op.  Errors: EINVAL, EUNSTABLE, EHIP, ENODEVICE.
 * NaN/Inf in the result are flagged on the device and reported by
 * dec_bpm_check_finite.  On a stream being captured into a HIP graph the
 * call launches one kernel per step (no persistent launch, no graph of its
 * own): the persistent launch's neighbour flags take values that grow from
 * call to call, which a replayed graph would not follow.
 */
int dec_bpm_propagate(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma, void* stream);

/*
 * dec_bpm_propagate without any allocation, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc): the
 * same steps, kernels and result as dec_bpm_propagate, but its two state
 * buffers and the persistent launch's flags live in a static device array of
 * 12 MiB that each device holds until the process ends, and every kernel is
 * launched directly (no graph is instantiated).  No hipMalloc, hipFree or
 * allocating library routine is called.  Limits: one-field handles with the
 * step tiles (EINVAL for rows of more than 12 neighbours, L^3 or L^4), and
 * 2 n_vert complex values of the handle's dtype at
 * most 12 MiB - 64 KiB (about 786k vertices in complex64, 393k in
 * complex128; EINVAL beyond, with the sizes in the message).  Every call on a
 * device shares that device's array, which keeps the last call's contents:
 * calls that overlap on one device (other streams, other threads, other
 * handles) race and must be serialised by the caller.  The flags are cleared
 * by a kernel at each call, so the call may be captured into a HIP graph
 * (persistent launch included) and the graph replayed.  Other errors as
 * dec_bpm_propagate.
 */
int dec_bpm_propagate_noalloc(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma, void* stream);

/*
 * The paper's unsplit scheme (Eq. 10 integrated as one ODE, "DEC beam
 * propagation"): n_steps classical RK4 steps of
 *   dPsi/dz = -i H_lin Psi + i gamma (M |Psi|^2) Psi - w Psi,
 * the Kerr term and the absorber evaluated inside every stage, at the fixed
 * step dz, in place on `field` (caller order).  Runs on the one-field step
 * tiles (one kernel per step); EINVAL for handles without them (the beta4
 * term, rows of more than 12 neighbours).  Other errors as dec_bpm_propagate.
 */
int dec_bpm_propagate_unsplit(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma, void* stream);

/*
 * The paper's integrator proper (section 3, the adaptive embedded Runge-Kutta
 * pair it runs through SciPy's RK45): Dormand-Prince 5(4) on the same
 * right-hand side as dec_bpm_propagate_unsplit, from z = 0 to z_end, first
 * trial step h0 (clipped to z_end), in place on `field` (caller order).
 * Error norm: the root mean square over vertices of
 * |e_p| / (atol + rtol max(|psi_p|, |psi'_p|)), e the embedded estimate; a
 * trial is accepted when it is below 1, and the next trial step is the last
 * one times min(10, max(0.2, 0.9 norm^(-1/5))), the growth capped at 1 right
 * after a rejection.  Trials, norms and decisions run on the device; the call
 * returns when the run has ended (it synchronises `stream`).
 * rtol >= 0 and atol > 0 (the paper's values are 1e-9 and 1e-11; complex64
 * handles need rtol of about 1e-6 or more, since rounding then dominates the
 * estimate).  max_attempts bounds accepted plus rejected trials.
 * n_accepted, n_rejected, last_h (the last accepted step) and z_reached may
 * be NULL.  Errors: EINVAL (arguments, or a handle without one-field step
 * tiles: the beta4 term, rows of more than 12 neighbours), EUNSTABLE (the
 * attempts ran out, or the step fell below 10 ulp of z, before z_end),
 * ENONFINITE (a non-finite error norm); in these cases `field` holds the last
 * accepted state and the counters are filled.  EHIP, ENODEVICE.  When the
 * handle's launch mode is the persistent one and every trial tile fits on the
 * device at once, the whole run is one cooperative launch; a tile whose wait
 * for the others exceeds the spin limit then ends the run with EHIP.  If the
 * runtime refuses the cooperative launch (it enqueues nothing then), the run
 * takes the per-trial kernels; dec_bpm_find_mode does the same with its
 * per-iteration kernels, and dec_bpm_time_kernels reports such a path as 0.
 */
int dec_bpm_propagate_adaptive(dec_bpm_t h, void* field, double z_end, double h0, double gamma, double rtol,
                               double atol, int64_t max_attempts, int64_t* n_accepted, int64_t* n_rejected,
                               double* last_h, double* z_reached, void* stream);

/*
 * Nonlinear eigenmode for a soliton launch (the stationary solutions
 * Psi(z) = phi e^{-i mu z} the paper launches in its soliton benchmark, whose
 * own solver is not given): mu phi = H_lin phi - gamma (M |phi|^2) phi at the
 * prescribed power P = sum_p H0_p |phi_p|^2 (the absorber plays no part).
 * Gradient flow with discrete normalisation: from phi_0 = field scaled to
 * power P, each iteration takes y = R4(-dtau A_k) phi_k (one classical RK4
 * step of dx/dtau = -A_k x, A_k = H_lin - gamma diag(M |phi_k|^2) frozen at
 * phi_k) and rescales y to power P.  Iteration k first evaluates
 * mu_k = Re<phi_k, A_k phi_k>_H0 / P and r_k = ||A_k phi_k - mu_{k-1} phi_k||_H0
 * / ||phi_k||_H0 (mu_{-1} = 0) and stops with phi_k when k > 0, tol > 0 and
 * r_k <= tol |mu_k|.  tol == 0 runs exactly max_iter iterations and returns
 * phi_{max_iter} (mu, r of the last tested iterate).  Converges to the mode
 * of lowest mu reachable from the start.  field (caller order) is the start
 * on entry and the mode on return; mu, residual, iterations (the k of the
 * result) may be NULL.  Synchronises `stream`.  One-field step tiles only
 * (EINVAL with the beta4 term or rows of more than 12 neighbours);
 * EUNSTABLE if dtau * rho(H_lin) exceeds the RK4 margin or if tol > 0 and
 * max_iter iterations did not converge (field then holds the last iterate),
 * ENONFINITE for a start without power or a non-finite iterate.
 */
int dec_bpm_find_mode(dec_bpm_t h, void* field, double power, double dtau, double gamma, double tol,
                      int64_t max_iter, double* mu, double* residual, int64_t* iterations, void* stream);

/* Synchronise `stream` and return ENONFINITE if the last propagate produced a
 * non-finite value, or a persistent launch's neighbour wait timed out (the
 * flag is cleared), else OK.  Not in the paper: a health check of the run. */
int dec_bpm_check_finite(dec_bpm_t h, void* stream);

/*
 * Diagnostics of a field (caller order), FP64 accumulation, synchronises:
 *   power       = sum_p H0_p |psi_p|^2 (conserved without absorber)
 *   hamiltonian = Psi^H H0 H_lin Psi - (gamma/2) sum_t chi_t |t| (mean_t |psi|^2)^2
 *                 (lumped: - (gamma/2) sum_p H0_p chibar_p |psi_p|^4).
 * Derived from Eq. 10-14 (not printed in the paper): the power is the
 * discrete L2 norm built from the Hodge star H0 that the semi-discrete flow
 * conserves, and the Hamiltonian satisfies i H0 dPsi/dz = dE/d conj(Psi) for
 * Eq. 10 with Eq. 14.  Either output pointer may be NULL.  Errors: EINVAL,
 * ENODEVICE, EHIP.
 */
int dec_bpm_diagnostics(dec_bpm_t h, const void* field, double gamma, double* power, double* hamiltonian,
                        void* stream);

/* H0-weighted inner product c = sum_p H0_p conj(a_p) b_p (the discrete L2
 * product of 0-forms through the Hodge star H0, "Discrete Hodge star"; derived:
 * the overlap objective of the gradient runs), conjugating its first argument,
 * FP64 accumulation; synchronises.  a, b: device complex vectors, caller order.
 * Errors: EINVAL, ENODEVICE, EHIP. */
int dec_bpm_overlap(dec_bpm_t h, const void* a, const void* b, double* re, double* im, void* stream);

/*
 * Checkpointed forward sweep and its adjoint (gradients of a real objective J
 * of the final field): the gradient loop of the structure optimisation the
 * paper motivates (Abstract, Conclusion).  The adjoint is derived here as the
 * exact reverse of the discrete Strang step built from Eq. 10-14 (the paper
 * gives no gradient formulation).  Gradients follow g = dJ/dRe + i dJ/dIm.
 * dec_bpm_workspace_size gives the bytes of caller-owned device workspace for
 * a run of n_steps with checkpoints every `every` steps (0 = ceil(sqrt(n))).
 * dec_bpm_forward_checkpointed propagates `field` in place like
 * dec_bpm_propagate and stores the checkpoints in the workspace.
 * dec_bpm_adjoint takes grad_out = dJ/dpsi(z_L) and, using the checkpoints of
 * the matching forward call (the forward call on this handle that last wrote
 * this workspace, with the same dz, n_steps, gamma and every, and an index
 * perturbation of the same values installed now as then; the handle keeps
 * the 64 most recent forward calls, one per workspace, so that several
 * forwards may precede their adjoints), returns
 * grad_field0 = dJ/dpsi(0) (complex, caller order) and, if grad_dn is not
 * NULL, grad_dn = dJ/d(dn) (double[n_vert], caller order).  Each segment
 * between checkpoints is recomputed forward, storing its stage vectors, then
 * swept backward.  On the one-kernel step tiles the forward call already
 * stores the last segment's stage vectors, so the adjoint call that follows
 * it recomputes every segment but that one; with every >= n_steps the workspace
 * holds the whole run (about five field vectors per step) and the adjoint
 * recomputes nothing, trading device memory for the recompute.  With a perfectly matched layer (complex L~ = H0~^{-1} K~)
 * the reverse sweep applies conj(L~) in the variables conj(H0~)^{-1} g (the
 * Kerr adjoint and the objective keep the real H0); both calls then need the
 * one-kernel step tiles, and a handle without them returns EINVAL.
 * Errors: EINVAL, EWORKSPACE, EUNSTABLE, EHIP.
 */
int dec_bpm_workspace_size(dec_bpm_t h, int64_t n_steps, int64_t every, size_t* bytes);
int dec_bpm_forward_checkpointed(dec_bpm_t h, void* field, double dz, int64_t n_steps, double gamma,
                                 int64_t every, void* workspace, size_t ws_bytes, void* stream);
int dec_bpm_adjoint(dec_bpm_t h, const void* grad_out, double dz, int64_t n_steps, double gamma, int64_t every,
                    void* workspace, size_t ws_bytes, void* grad_field0, double* grad_dn, void* stream);

/*
 * Batched propagation of many launch fields on many meshes at once (the
 * paper's use case of sweeping fibre cross-sections and launch conditions,
 * Abstract and Conclusion; each field follows Eq. 10 exactly as
 * dec_bpm_propagate would advance it alone).  All meshes must share dtype,
 * p1, beta4 and nonlinearity mode, and none may carry a PML, L^3, L^4 or a
 * non-Kerr response.  fields_per_mesh[m] (1 to 4096) is the number of fields
 * on mesh m; counts may differ between meshes.  The packed field layout is
 * field-minor, per mesh in the order given: element (mesh m, caller vertex i,
 * field f < F_m) sits at complex offset base_m + i * F_m + f, with
 * base_m = n_0 F_0 + ... + n_{m-1} F_{m-1}.  The batch holds its own copy of
 * the operators; the mesh handles may be destroyed afterwards; the host array
 * fields_per_mesh is copied.  Errors: EINVAL (NULL or bad arguments, meshes
 * that do not match), ENOMEM, EHIP.
 */
int dec_bpm_batch_create(const dec_bpm_t* meshes, int32_t n_meshes, const int32_t* fields_per_mesh,
                         dec_bpm_batch_t* out);
/* Releases the batch's device memory (NULL is a no-op). */
void dec_bpm_batch_destroy(dec_bpm_batch_t b);
/* Total packed complex elements (sum_m n_m * fields_per_mesh[m]).  Errors: EINVAL. */
int dec_bpm_batch_size(dec_bpm_batch_t b, int64_t* n_elems);
/* n_steps Strang steps of length dz of every field, in place in the packed
 * layout above (caller-owned device memory, dec_bpm_batch_size elements);
 * the same scheme and arguments as dec_bpm_propagate (Eq. 10-14), each field
 * on its own mesh.  Errors: EINVAL, EUNSTABLE, EHIP, ENODEVICE (a batch of
 * host-only meshes).  Non-finite results are flagged on the device and
 * reported by dec_bpm_batch_check_finite. */
int dec_bpm_batch_propagate(dec_bpm_batch_t b, void* packed_fields, double dz, int64_t n_steps, double gamma,
                            void* stream);
/* As dec_bpm_check_finite, for a batch. */
int dec_bpm_batch_check_finite(dec_bpm_batch_t b, void* stream);

/*
 * Launch tuning (not in the paper: how the same arithmetic is scheduled on the
 * device; no call here changes a result beyond rounding order, and the
 * one-kernel and persistent split steps give identical bits).
 * dec_bpm_autotune times candidate launch shapes (unfused:
 * block size; fused LDS-tiled path: threads per tile; both: z steps per
 * hipGraph and the XCD-aware block mapping) on the handle's own work buffers
 * with HIP events and keeps the fastest; the result is cached in the JSON file
 * named by DEC_BPM_TUNE_CACHE if that variable is set.  Synchronises.
 * Fused paths of one-field handles: fused = 1 (without the beta4 term) runs
 * two kernels per z step (stages 2+3, and stage 4 + Kerr/absorber + next
 * stage 1, each on a tile of rows with three halo rings in LDS); fused = 2
 * runs the whole z step (four stages + Kerr/absorber) as one kernel on tiles
 * with five halo rings (four for the lumped nonlinearity; with the beta4 term
 * two rings per stage: nine, or eight); fused = 3 (without the beta4 term)
 * runs a whole propagate in one persistent launch on those tiles, every tile
 * resident with its operator rows in registers, tiles synchronising with their
 * neighbour tiles only (available when all tiles fit on the device at once;
 * otherwise, and with the beta4 term, fused = 3 runs as fused = 2).  The
 * persistent launch is an ordinary one (about 12 us less per call than a
 * cooperative launch): its workgroups are all resident once earlier work on
 * the device has drained, and persistent launches of this process on
 * different streams are ordered one after another.  Work that keeps compute
 * units busy for longer than the wait bound (another process's persistent
 * kernel, say) can make it give up; DEC_BPM_COOPERATIVE=1 in the environment
 * at handle creation selects the cooperative launch, whose residency the
 * runtime guarantees.  A handle that has no tiles for the requested mode runs
 * the unfused kernels.  A persistent neighbour wait that exceeds its bound
 * (DEC_BPM_SPIN_LIMIT polls, default 2^20, of the order of a second) leaves the launch
 * early and makes the next dec_bpm_check_finite report DEC_BPM_ENONFINITE.
 * In complex64 the persistent split step keeps its per-slot buffers at fixed
 * offsets in static LDS (tiles of at most 2432 slots); DEC_BPM_FIXED_LDS=0 in
 * the environment (read once per process) selects the runtime-sized layout,
 * with the same results bit for bit.
 */
typedef struct {
  int32_t block_size;       /* threads per workgroup of the unfused kernels      */
  int32_t steps_per_graph;  /* z steps per captured hipGraph (1 = no graph)      */
  int32_t fused;            /* 0 unfused, 1 two tile kernels, 2 one kernel per    */
                            /* step, 3 persistent launch                          */
  int32_t tile_block;       /* threads per workgroup of the fused kernels        */
  int32_t xcd_remap;        /* 1: consecutive row blocks on one XCD               */
} dec_bpm_tuning;
int dec_bpm_autotune(dec_bpm_t h, double dz, double gamma, void* stream);
int dec_bpm_batch_autotune(dec_bpm_batch_t b, double dz, double gamma, void* stream);
int dec_bpm_get_tuning(dec_bpm_t h, dec_bpm_tuning* t);
int dec_bpm_set_tuning(dec_bpm_t h, const dec_bpm_tuning* t);
/* Batched engines: `fused` selects the LDS-tiled batched kernels (one halo
 * ring, all fields of a tile staged in LDS) over the row-parallel ones. */
int dec_bpm_batch_get_tuning(dec_bpm_batch_t b, dec_bpm_tuning* t);
int dec_bpm_batch_set_tuning(dec_bpm_batch_t b, const dec_bpm_tuning* t);

/*
 * Per-kernel timing (measurement support, not in the paper) with HIP events on
 * `stream`: each kernel class is
 * captured `reps` times back to back in a hipGraph and timed; the mean device
 * time per launch in milliseconds goes to ms[DEC_BPM_NUM_KERNELS] and the
 * algorithmic bytes one launch moves to bytes[DEC_BPM_NUM_KERNELS] (either may
 * be NULL; classes a handle does not use report 0).  Synchronises.
 */
enum {
  DEC_BPM_K_KERR = 0,     /* fused Kerr phase + absorber (M gather)               */
  DEC_BPM_K_STAGE = 1,    /* RK4 stage: L gather + stage update                   */
  DEC_BPM_K_LAP = 2,      /* bare L application (first half of a beta4 stage)    */
  DEC_BPM_K_TILE_A = 3,   /* fused tile kernel: stage 4 + Kerr/absorber + stage 1 */
  DEC_BPM_K_TILE_B = 4,   /* fused tile kernel: stages 2 + 3                      */
  DEC_BPM_K_STEP = 5,     /* one-kernel z step: four stages + Kerr/absorber       */
  DEC_BPM_K_PERSIST = 6,  /* persistent launch of max(reps, 2000) steps: per step */
  DEC_BPM_K_UNSPLIT = 7,  /* one unsplit RK4 step (dec_bpm_propagate_unsplit)     */
  DEC_BPM_K_DP5 = 8,      /* one adaptive Dormand-Prince trial (seven stages)     */
  DEC_BPM_K_MODE = 9,     /* one nonlinear mode iteration (dec_bpm_find_mode)     */
  DEC_BPM_K_DP5_PERSIST = 10, /* one trial inside a persistent adaptive launch of   */
                              /* max(reps, 200) trials (0: the trial tiles do not   */
                              /* all fit on the device at once)                     */
  DEC_BPM_K_MODE_PERSIST = 11, /* one iteration inside a persistent mode-solver     */
                               /* launch of max(reps, 200) iterations (0: not used  */
                               /* by this handle)                                   */
  DEC_BPM_K_UNSPLIT_PERSIST = 12, /* one unsplit RK4 step inside a persistent launch */
                                  /* of max(reps, 2000) steps (0: not used)          */
  DEC_BPM_NUM_KERNELS = 13
};
int dec_bpm_time_kernels(dec_bpm_t h, double dz, double gamma, int32_t reps, double* ms, double* bytes,
                         void* stream);
int dec_bpm_batch_time_kernels(dec_bpm_batch_t b, double dz, double gamma, int32_t reps, double* ms,
                               double* bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DEC_BPM_H */
