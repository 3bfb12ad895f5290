// Device data layout and kernel launchers of the DEC beam-propagation library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace decbpm {

// Rows are vertices in device order (a Hilbert curve per mesh; meshes of a
// batch are concatenated).  Every row carries F fields stored field-minor:
// the complex value of (row r, field f) sits at r * F + f.
//
// The operators are stored as sliced ELL with slices of 64 rows (one
// wavefront): slice s keeps width W_s = max off-diagonal degree of its rows,
// and entry k of row r lives at off_s + k * 64 + (r & 63), so lane j of a
// wavefront reading entry k touches consecutive words.  One 64-bit word per
// slice packs sl_info[s] = (off_s << 8) | W_s.  Only off-diagonal neighbours
// are stored; L is applied in difference form
//   (L x)_p = sum_q c_pq (x_p - x_q),   c_pq = -K_pq / H0_p,
// which makes L 1 = 0 exact in floating point.  Padding entries point at the
// row itself with zero weights.
template <typename T>
struct DevOps {
  int64_t n_rows;      // rows (vertices summed over meshes)
  int32_t F;           // fields per row
  int32_t lgF;         // log2(F) when F is a power of two, else -1
  int32_t wmax;        // largest slice width
  const int64_t* sl_info;
  const int32_t* col;  // device-order neighbour
  const T* lw;         // c_pq
  const T* mw;         // M_pq (off-diagonal), nullptr for the lumped nonlinearity
  const T* mdiag;      // M_pp
  const T* v;          // vertex potential (+ index perturbation)
  const T* w;          // absorber strength
  const double* h0;    // dual areas (device order)
  T p1, beta4;
  int32_t xcd_remap;   // 1: map consecutive row blocks onto one XCD
  int32_t nk;          // Kerr response: 0 N(I) = I, 1 saturable I/(1 + I/npar), 2 cubic-quintic I - npar I^2
  T npar;
};

// Tiles for the fused kernels (one field per row, no beta4 term).  Tile t
// owns the contiguous device rows [t*TS, t*TS + nT) and carries its halo
// rings H1, H2, H3 (rows adjacent to the previous rings).  Inside a tile every
// row is a "slot": slots [0, nT) are the owned rows in order, then H1, H2, H3
// (global rows listed in ext).  The operator rows of slots in T, H1 and H2 are
// stored again with 16-bit slot-local columns, sliced by 64 slots like the
// global operator (lsl holds (offset << 8) | width per slice, offsets
// relative to ent_base[t]).
template <typename T>
struct TileOps {
  int32_t n_tiles;
  int32_t TS;
  int32_t max_slots;        // largest slot count of a tile (all rings), LDS sizing
  int32_t max_compute;      // largest count of slots with operator rows
  const int32_t* hdr;       // [n_tiles * hdr_stride].  Classic layout (stride 8): ring counts nT,
                            // nH1..nH3, ext base, slice-table base.  Step layout (stride 16):
                            // cumulative slot counts of rings 0..k for k = 0..9, [15] = ring count
  const int64_t* ent_base;  // [n_tiles]
  const int32_t* ext;       // halo rows (device order)
  const int32_t* lsl;
  const uint16_t* lcol;
  const T* llw;
  const T* lmw;             // nullptr for the lumped nonlinearity
  const T* llwi;            // imaginary part of the L weights (complex-stretched L), else nullptr
  const uint8_t* dep;       // step layout: per slot (ext stride), an owned row's graph distance to
                            // the nearest row the tile does not own (capped at 7); 0 for halo slots
  int32_t ext_stride;       // step layout: per-tile stride of ext (every slot listed) and of lsl;
  int32_t lsl_stride;       // 0: classic layout (offsets in the header, ring 0 implicit)
  int32_t hdr_stride;       // ints per tile header (8 classic, 16 step layout)
};

enum FusedKind { FUSED_S4_NL_S1 = 0, FUSED_S2_S3 = 1, FUSED_NL_S1 = 2, FUSED_S4_NL = 3 };

template <typename T>
struct Cplx;
template <>
struct Cplx<float> {
  using type = float2;
};
template <>
struct Cplx<double> {
  using type = double2;
};
template <typename T>
using cplx_t = typename Cplx<T>::type;

// ---- launchers (asynchronous on `st`) ----
// y = psi + coef * A x with A = -i (p1 L - diag v) (beta4 == 0) or, when t = L x
// is given, A = -i (p1 L + beta4 L^2 - diag v).  If s_out is non-null it
// receives |y|^2 phi(w, tau_s) for the next Kerr substep.  y may alias psi.
template <typename T>
void launch_stage(const DevOps<T>& d, const void* x, const void* t, const void* psi, void* y, double coef,
                  void* s_out, double tau_s, int block, hipStream_t st);
// t = L x
template <typename T>
void launch_lap(const DevOps<T>& d, const void* x, void* t, int block, hipStream_t st);
// y = a L z + b x  (one Horner step of a sum of powers of L; F = 1)
template <typename T>
void launch_lapc(const DevOps<T>& d, const void* z, const void* x, double a, double b, void* y, int block,
                 hipStream_t st);
// s = |psi|^2 phi(w, tau)
template <typename T>
void launch_prep_s(const DevOps<T>& d, const void* psi, void* s, double tau, int block, hipStream_t st);
// psi_out <- psi_in e^{-w tau} exp(i gamma (M s)); s gathered; psi_out may alias psi_in
template <typename T>
void launch_kerr(const DevOps<T>& d, const void* psi_in, void* psi_out, const void* s, double tau, double gamma,
                 int block, hipStream_t st);
// dst[r*F+f] = src[perm[r]*F+f] (caller order -> device order), optionally scaled by 1/h0
template <typename T>
void launch_perm_in(const DevOps<T>& d, const int32_t* perm, const void* src, void* dst, int scale_inv_h0, int block,
                    hipStream_t st);
// dst[perm[r]*F+f] = src[r*F+f] (device order -> caller order), optionally scaled by h0;
// a non-finite value sets *flag (if flag is non-null)
template <typename T>
void launch_perm_out(const DevOps<T>& d, const int32_t* perm, const void* src, void* dst, int scale_h0, int* flag,
                     int block, hipStream_t st);
// x[:] = re + i im
template <typename T>
void launch_fill(const DevOps<T>& d, void* x, double re, double im, int block, hipStream_t st);
// power and Hamiltonian (F = 1): per-block FP64 partials, then one fixed-order block
template <typename T>
void launch_diag(const DevOps<T>& d, const void* psi, double gamma, double* partials, int n_blocks, double* out,
                 hipStream_t st);
// overlap sum_j h0c_j conj(a_j) b_j over caller order
template <typename T>
void launch_overlap(int64_t n, const double* h0c, const void* a, const void* b, double* partials, int n_blocks,
                    double* out, hipStream_t st);
// n complex values src -> dst
template <typename T>
void launch_copy(int64_t n, const void* src, void* dst, int block, hipStream_t st);
// y = p1 t + beta4 t2 - v x  (t = L x, t2 = L t; t2 may be null when beta4 == 0)
template <typename T>
void launch_hcombine(const DevOps<T>& d, const void* x, const void* t, const void* t2, void* y, int block,
                     hipStream_t st);
// v[r] = v0[r] + (dn ? dn[perm[r]] : 0)
template <typename T>
void launch_set_v(int64_t n, const T* v0, const double* dn, const int32_t* perm, T* v, int block, hipStream_t st);

// ---- adjoint (F = 1), in H0-scaled adjoint variables lambda = H0^{-1} g ----
// One link of the reverse Horner chain of an RK4 step:
//   u_out = coef * A u_in   (A as in launch_stage; t = L u_in when beta4 != 0)
//   acc   = (init ? u_in : acc) + u_out
//   gdn  += cdn * h0 * Re(i conj(u_in) yf)
// u_out may be null (last link).
template <typename T>
void launch_adj_stage(const DevOps<T>& d, const void* u_in, const void* t, void* u_out, void* acc, int init,
                      const void* yf, double coef, double cdn, double* gdn, int block, hipStream_t st);
// sm = (|psi_in|^2 phi(w,tau), gamma Re(i conj(lam_out) psi_out)) per row
template <typename T>
void launch_adj_prep(const DevOps<T>& d, const void* psi_in, const void* psi_out, const void* lam_out, void* sm,
                     double tau, double gamma, int block, hipStream_t st);
// lam_in = conj(E) lam_out + 2 phi psi_in (M mu),  E = e^{-w tau} e^{i gamma M s}
template <typename T>
void launch_adj_kerr(const DevOps<T>& d, const void* psi_in, const void* lam_out, const void* sm, void* lam_in,
                     double tau, double gamma, int block, hipStream_t st);
// Fused z-step kernels on tiles (see TileOps):
//   FUSED_S4_NL_S1: psi_new = psi + h A y3 (rings <= 2), psi'' = NL_tau(psi_new) (rings <= 1),
//                   y1 = psi'' + h/4 A psi'' (owned rows); writes psi'' -> out_psi, y1 -> out_y
//   FUSED_S2_S3:    y2 = psi + h/3 A y1 (rings <= 1), y3 = psi + h/2 A y2; writes y3 -> out_y
//   FUSED_NL_S1:    first step: psi'' = NL_tau(psi), y1 = psi'' + h/4 A psi''
//   FUSED_S4_NL:    last step: psi_new = psi + h A y3, psi'' = NL_tau(psi_new)
// in_x is y3 (S4 kinds), y1 (S2_S3) or unused; in_psi is the state psi.
// Batched (F > 1) stage / Laplacian / Kerr kernels on one-ring tiles whose
// fields are staged in LDS (same arithmetic as launch_stage/lap/kerr).
template <typename T>
void launch_bstage(const DevOps<T>& d, const TileOps<T>& tl, const void* x, const void* t, const void* psi, void* y,
                   double coef, void* s_out, double tau_s, hipStream_t st);
template <typename T>
void launch_blap(const DevOps<T>& d, const TileOps<T>& tl, const void* x, void* t, hipStream_t st);
template <typename T>
void launch_bkerr(const DevOps<T>& d, const TileOps<T>& tl, const void* psi_in, void* psi_out, const void* s,
                  double tau, double gamma, hipStream_t st);

// One kernel per merged Strang step on tiles with five halo rings (hdr holds
// the six ring counts in [0..5], the ext and slice-table bases in [6], [7]):
// out_psi = NL_tau(LIN_h(in_psi)) on the owned rows.  With out_perm the result
// goes to out_psi[out_perm[r]] (the caller's order) and a non-finite value
// sets bit 0 of *flag.
template <typename T>
void launch_step(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, double h, double tau,
                 double gamma, int block, hipStream_t st, const int32_t* out_perm = nullptr, int* flag = nullptr);
// One whole z step with the beta4 L^2 term (two gathers per stage) on tiles of
// 8 halo rings (9 with the triangle-averaged Kerr term); out_perm as above.
template <typename T>
void launch_step_b4(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, double h,
                    double tau, double gamma, int block, hipStream_t st, const int32_t* out_perm = nullptr,
                    int* flag = nullptr);
// Batched fields between the caller's layout (per mesh, field-minor, that
// mesh's own field count) and the device's (row * F + f, F fields per row):
// device element (row, f) is caller element cbase[row] + f when
// f < fcount[row]; other device fields are zero in (out = false) and dropped
// out (out = true, which also sets bit 0 of *flag for a non-finite value).
// field_major: the device layout is field f of row r at f * n_rows + r
// instead of r * F + f.
template <typename T>
void launch_bperm(const DevOps<T>& d, const int64_t* cbase, const int32_t* fcount, const void* src, void* dst,
                  bool out, int* flag, int block, hipStream_t st, bool field_major = false);
// Every field of a batch (d.F fields, field-major device layout) on one-field
// step tiles: one merged z step (LIN(h) then NL(tau)), and NL(tau) alone.
// One workgroup per tile steps the fields one after another with the
// operator rows kept in registers.
template <typename T>
void launch_step_fields(const DevOps<T>& d, const TileOps<T>& tl, const void* in, void* out, double h, double tau,
                        double gamma, int block, hipStream_t st);
template <typename T>
void launch_kerr_fields(const DevOps<T>& d, const TileOps<T>& tl, const void* in, void* out, double tau,
                        double gamma, int block, hipStream_t st);
// NL(tau) of the caller's field (caller order: row r at src[perm[r]]) into
// the device-order buffer dst, on the step tiles (any ring count): the first
// half step of a propagate, with the persistent launch's per-row arithmetic.
template <typename T>
void launch_kerr_tile(const DevOps<T>& d, const TileOps<T>& tl, const void* src, const int32_t* perm, void* dst,
                      double tau, double gamma, int block, hipStream_t st);
// One RK4 stage of the operator sum with terms up to p4 L^4 on tiles of D
// halo rings (D = 4 with p4, else 3): out = base + coef (-i)(sum_n p_n L^n x
// - V x) on the owned rows (p1 and p2 = beta4 from d), by Horner in LDS; with
// s_out also the Kerr substep's integral of |out|^2 over tau_s.
template <typename T>
void launch_hstage(const DevOps<T>& d, const TileOps<T>& tl, const void* x, const void* base, void* out, double coef,
                   double p3, double p4, void* s_out, double tau_s, int block, hipStream_t st);
// One step of classical RK4 on the whole right-hand side (the Kerr term and
// the absorber inside every stage) on the five-ring step tiles (four rings are
// used: one per stage).
template <typename T>
void launch_unsplit(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, double h,
                    double gamma, int block, hipStream_t st);

// Device-resident state of an adaptive Dormand-Prince 5(4) run.  A trial
// kernel reads the state from x[cur], writes the fifth-order candidate to
// x[1 - cur], and its last-finishing workgroup accepts (cur flips, z advances)
// or rejects and sets the next trial step.  Once done is set, trials return
// at once.
struct Dp5Ctl {
  double z, z_end;    // accepted position, end of the run
  double h_abs;       // step size before clipping to z_end
  double h_step;      // the trial step of the next attempt (clipped)
  double z_trial;     // z + h_step
  double last_h;      // last accepted step
  double err;         // error norm of the last attempt
  double facmax;      // largest growth factor after an accepted step
  int64_t accepted, rejected, max_attempts;
  int32_t cur, prev_rejected, done;
  int32_t status;  // 0 running or reached z_end, 1 attempts exhausted, 2 non-finite error, 3 step underflow
};

// Sets up an adaptive run: z = 0, first trial step min(h0, z_end), cur = 0,
// arrival count 0; done at once when z_end == 0.
void launch_dp5_init(Dp5Ctl* ctl, uint32_t* arrivals, double z_end, double h0, int64_t max_attempts, double facmax,
                     hipStream_t st);
// One trial step of the pair and its accept/reject decision on the seven-ring
// tiles of tl (one ring per stage).  partial: n_tiles doubles of scratch;
// inv_n: 1 / vertex count (the norm is a mean over vertices).
template <typename T>
void launch_dp5(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, Dp5Ctl* ctl, double* partial,
                uint32_t* arrivals, double gamma, double rtol, double atol, double inv_n, int block, hipStream_t st);

// Device-resident state of a nonlinear mode iteration (imaginary-z RK4 with
// the nonlinearity frozen per step, renormalised to the power P): the current
// iterate is s * x[cur].  Once done is set, iterations return at once.
struct ModeCtl {
  double s;        // scale of x[cur] giving the current iterate
  double power;    // prescribed power P = sum_p H0_p |phi_p|^2
  double mu_prev;  // Rayleigh quotient of the previous iterate (0 before the first)
  double mu, res;  // quotient and residual of the last tested iterate
  double tol;      // stop when r <= tol |mu| (k > 0); 0: run max_iter steps
  int64_t iter, max_iter;  // index k of the current iterate
  int32_t cur, done;
  int32_t status;  // 0 converged (or max_iter reached with tol == 0), 1 not converged, 2 non-finite
  int32_t pad;
};

// Starts the iteration from x[0]; pw[0] holds the power of x[0].
void launch_mode_init(ModeCtl* ctl, uint32_t* arrivals, const double* pw, double power, double tol, int64_t max_iter,
                      hipStream_t st);
// One iteration and its stopping test on the step tiles (rings 0..4 staged);
// partial: 4 * n_tiles doubles of scratch.
template <typename T>
void launch_mode(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, ModeCtl* ctl, double* partial,
                 uint32_t* arrivals, double h, double gamma, int block, hipStream_t st);
// The adaptive run to its end in one cooperative launch with every
// seven-ring tile resident (a wait timeout sets status bit 2 and leaves the
// controller state not done); partial: 2 * n_tiles doubles, flags: n_tiles
// ints of scratch (cleared by the launch).
template <typename T>
int dp5_persist_capacity(const DevOps<T>& d, const TileOps<T>& tl, int block);
template <typename T>
hipError_t launch_dp5_persist(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, Dp5Ctl* ctl,
                              double* partial, int32_t* flags, int32_t* status, int32_t spin_limit, double gamma,
                              double rtol, double atol, double inv_n, int block, hipStream_t st);
// The mode iteration to its end (stopping test, max_iter or a wait timeout:
// status bit 2) in one cooperative launch with every step tile resident;
// flags: n_tiles ints of scratch (cleared by the launch).
// mode_persist_capacity: resident workgroups at `block` threads.
template <typename T>
int mode_persist_capacity(const DevOps<T>& d, const TileOps<T>& tl, int block);
template <typename T>
hipError_t launch_mode_persist(const DevOps<T>& d, const TileOps<T>& tl, void* x0, void* x1, ModeCtl* ctl,
                               double* partial, int32_t* flags, int32_t* status, int32_t spin_limit, double h,
                               double gamma, int block, hipStream_t st);
// x[0..n) *= s (complex, device order)
template <typename T>
void launch_scale(int64_t n, void* x, double s, int block, hipStream_t st);

// The one-kernel step that also writes the owned rows' stage vectors y1..y3
// and the state before the Kerr substep (the adjoint's forward recompute).
template <typename T>
void launch_step_rec(const DevOps<T>& d, const TileOps<T>& tl, const void* in_psi, void* out_psi, void* y1, void* y2,
                     void* y3, void* b, double h, double tau, double gamma, int block, hipStream_t st);
// One reverse z step of the adjoint on the step tiles (lam_out must not alias
// lam_in; gdn accumulates in place).  sig: H0~ / H0 per row (device order) for
// tiles with complex L weights (a perfectly matched layer), else unused.
template <typename T>
void launch_step_adj(const DevOps<T>& d, const TileOps<T>& tl, const void* lam_in, const void* fa, const void* fb,
                     const void* y3, const void* y2, const void* y1, const void* fa0, void* lam_out, double* gdn,
                     double h, double tau, double gamma, const void* sig, int block, hipStream_t st);

// Where a persistent launch takes its state from and puts its result.
// in: the caller's field (caller order, row r at in[perm[r]]); the launch
//     starts with NL(tau_first) of it (split-step body only).  nullptr: the
//     state before the first step is already in buf0 (device order).
// out: the caller's field for the result (caller order); the last step then
//     uses NL(tau_last) and writes there, setting bit 0 of *status for a
//     non-finite value.  nullptr: every step is a merged step (NL(h)) and the
//     result stays in buf0/buf1 (buf0 after an even step count).
// out may alias in.  base: a value no flag exceeds before the launch; the
// launch publishes base + 1, base + 2, ... (at most base + n_steps + 1).
struct PersistIO {
  const void* in = nullptr;
  void* out = nullptr;
  const int32_t* perm = nullptr;
  int32_t base = 0;
  double tau_first = 0.0, tau_last = 0.0;
};

// Persistent z stepping (n_steps steps in one launch, one resident
// workgroup per tile of the five-ring step tiles).  nb_ptr/nb_list: per tile,
// the other tiles owning its halo rows.  flags: n_tiles ints that only grow
// (see PersistIO::base).  status: bit 1 is set if a neighbour wait timed out.
// coop: a cooperative launch (the runtime guarantees that every workgroup is
// resident at once, and fails the launch otherwise); else an ordinary launch
// of a grid that persist_capacity says fits, whose workgroups all become
// resident once earlier work on the device has drained (the bounded waits
// cover the time until then).  persist_capacity: resident workgroups the
// device holds for this kernel at `block` threads (0 if the tiles do not fit
// the kernel).  body: 0 the merged split step (LIN(h) then NL(h)), 1 one
// unsplit RK4 step of the whole right-hand side.
template <typename T>
int persist_capacity(const DevOps<T>& d, const TileOps<T>& tl, int block, int body = 0);
template <typename T>
hipError_t launch_persist(const DevOps<T>& d, const TileOps<T>& tl, const int32_t* nb_ptr, const int32_t* nb_list,
                          void* buf0, void* buf1, int32_t* flags, int32_t* status, int32_t n_steps,
                          int32_t spin_limit, double h, double gamma, int block, hipStream_t st, int body,
                          const PersistIO& io, bool coop = true);
// n ints set to 0
void launch_zero_i32(int64_t n, int32_t* x, hipStream_t st);

// out_rec (may be null) receives, for owned rows, y2 (FUSED_S2_S3) or the
// state before the Kerr substep (S4 kinds): the adjoint's segment recompute.
template <typename T>
void launch_fused(const DevOps<T>& d, const TileOps<T>& tl, int kind, const void* in_x, const void* in_psi,
                  void* out_psi, void* out_y, void* out_rec, double h, double tau, double gamma, int block,
                  hipStream_t st);
// Fused adjoint of one z step on tiles (lambda = H0^{-1} g variables):
//   kind 1: vin = lambda after the step, fa = a_n (state after the Kerr substep),
//           fb = b_n (state before it), y3, y2, y1 = the step's stage vectors;
//           writes out_u = u2, acc = lam_b + u1 + u2, gdn += link 1-3 terms.
//   kind 2: vin = u2, fa = a_{n-1} (the step's input state), acc as written by kind 1;
//           writes out_u = lambda before the step, gdn += link 4 term.
template <typename T>
void launch_fused_adj(const DevOps<T>& d, const TileOps<T>& tl, int kind, const void* vin, const void* fa,
                      const void* fb, const void* y3, const void* y2, const void* y1, void* out_u, void* acc,
                      double* gdn, double h, double tau, double gamma, int block, hipStream_t st);

// out[perm[r]] = gdn[r]
void launch_gdn_out(int64_t n, const int32_t* perm, const double* gdn, double* out, int block, hipStream_t st);
void launch_zero_f64(int64_t n, double* x, int block, hipStream_t st);

}  // namespace decbpm
