/*
 * iobm.h -- C ABI of libiobm, the MI355X (gfx950) scattering-state solver of
 * the improved overbridging-boundary-matching (IOBM) method with FFT-applied
 * jellium self-energies and preconditioned conjugate gradients
 * (Egami, Hirose, Ono, "Novel time-saving first-principles calculation
 * method for electron-transport properties", arXiv:1009.5300).
 *
 * Problem (Sec. II, Eqs. (1)-(8)): on an nx x ny x nz real-space grid that
 * is periodic in x and y (lateral Bloch vector kappa = 0) and truncated
 * along z (the transport axis), solve for every requested energy E and
 * incident lateral channel mu
 *
 *     [E - H_T - Sigma_L(E) - Sigma_R(E)] psi = b_mu(E)                (Eq. 6)
 *
 * where H_T = -1/2 Laplacian (central FD of order 2*nf, Eq. (1)) + V(r)
 * [+ separable nonlocal term], Sigma_L/R are the retarded self-energies of
 * two semi-infinite jellium electrodes (V = 0, same stencil), acting on the
 * first/last nf planes and diagonal in the lateral plane waves (Eqs. (14)-
 * (15); N_f x N_f per mode for nf > 1), and b_mu carries the unit-amplitude
 * incident Bloch wave of channel mu.  Transmission and reflection are read
 * off psi at the boundary planes (scattering condition, Eq. (7)).
 *
 * Conventions
 *  - Hartree atomic units (hbar = m = 1); energies measured from the lead
 *    band bottom (the jellium potential is 0).
 *  - Flat voxel index (k*ny + j)*nx + i; x fastest; k = plane 0..nz-1.
 *    Plane 0 faces the left electrode, plane nz-1 the right one.
 *  - Complex arrays are interleaved (re, im).  complex128 = 2 doubles,
 *    complex64 = 2 floats.
 *  - Lateral channel id m = iy*nx + ix, ix/iy in FFT order
 *    (nu_x = ix for ix < nx/2, else ix - nx); lateral plane wave
 *    exp(2 pi i (nu_x i / nx + nu_y j / ny)).
 *  - Lateral Fourier transform normalised as in Eq. (16): psi~_nu =
 *    (1/Nxy) sum_l exp(-i G_nu . r_l) psi(r_l).
 *  - An incident wave has unit amplitude on its lateral plane wave at plane 0.
 *    t[nu][mu] is the amplitude of outgoing channel nu at plane nz-nf,
 *    r[nu][mu] the reflected amplitude at plane 0; T_mu = sum_nu
 *    (v_nu/v_mu) |t_nu,mu|^2 over open nu, R_mu likewise (Landauer-Buttiker,
 *    Sec. III).
 *
 * Ownership and streams
 *  - The caller owns every buffer it passes.  Pointers documented "device"
 *    must be device memory on the context's device (e.g. torch tensors);
 *    "host" pointers are ordinary host memory.
 *  - The context owns its copies of V, the nonlocal data, per-energy mode
 *    tables and all solver workspaces; iobm_destroy frees them.
 *  - All device work is enqueued on the stream given to iobm_create (NULL =
 *    the null stream).  Calls that return host results synchronise that
 *    stream before returning (iobm_precondition when it returns r^T z);
 *    iobm_apply and iobm_precondition otherwise do not.
 *  - A context is not thread-safe; separate contexts are independent.
 *
 * Errors
 *  - Every call returns an iobm_status; no C++ exception crosses the ABI.
 *    Arguments are validated before any launch.  iobm_last_error(ctx) holds
 *    a message for the last failure on that context.
 */
#ifndef IOBM_H
#define IOBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct iobm_ctx_s* iobm_ctx;

typedef enum {
  IOBM_OK = 0,
  IOBM_E_INVALID_ARG = 1,   /* bad size, pointer, option, channel id, or non-finite input */
  IOBM_E_BAD_STATE = 2,     /* e.g. solve before iobm_set_potential */
  IOBM_E_OOM = 3,           /* device allocation failed */
  IOBM_E_DEVICE = 4,        /* HIP runtime error (message in iobm_last_error) */
  IOBM_E_NOT_CONVERGED = 5, /* some right-hand side missed the tolerance; results of
                               converged ones are valid, per-RHS status in the stats */
  IOBM_E_BREAKDOWN = 6,     /* Krylov breakdown that restarts could not cure */
  IOBM_E_AT_THRESHOLD = 7,  /* energy within 1e-9 (relative) of a lateral channel threshold */
  IOBM_E_UNSUPPORTED = 8    /* valid request the library does not implement */
} iobm_status;

/* Grid: nx, ny >= 2 (lateral, periodic), nz >= 2*nf (planes of the transition
 * region, both boundary plane groups included), spacings > 0 in bohr,
 * nf in {1, 2, 3} = half width of the central FD stencil (Eq. (1)). */
typedef struct {
  int32_t nx, ny, nz;
  double hx, hy, hz;
  int32_t nf;
} iobm_grid;

enum { IOBM_C128 = 0,          /* complex128 throughout */
       IOBM_C64_REFINED = 1 }; /* complex64 inner COCG, FP64 residual + refinement */

enum { IOBM_PC_NONE = 0,
       IOBM_PC_TRUNCATED_LAPLACIAN = 1, /* Eq. (17): C0 g + C1 sum over the 6 face
                                           neighbours, C0 = 1, C1 = exp(-alpha) */
       IOBM_PC_LATERAL_FFT = 2,         /* exact inverse of the V = 0 operator: lateral
                                           FFT + per-mode z Green's function */
       IOBM_PC_JACOBI = 3 };            /* diagonal scaling (Sec. II): z = r / diag A(E),
                                           diag A = E - V - kinetic diagonal - nonlocal
                                           diagonal - real-space Sigma diagonal on the
                                           face planes */

typedef struct {
  int32_t precision;   /* IOBM_C128 or IOBM_C64_REFINED */
  int32_t precond;     /* IOBM_PC_* */
  double alpha;        /* Eq. (17) parameter, C1 = exp(-alpha); default 1.8 */
  double tol;          /* stop when ||b - A psi||_2 <= tol ||b||_2 (FP64); default 1e-10 */
  double inner_tol;    /* IOBM_C64_REFINED: reliable-update factor; the complex64
                          residual is replaced by the FP64 true residual (and the
                          correction folded into psi) each time it has fallen by
                          this factor; default 1e-3 */
  int32_t max_iter;    /* total COCG iterations per RHS; default 50000 */
  int32_t side;        /* 0: incidence from the left electrode, 1: from the right */
  int32_t check_every; /* iterations between host convergence checks; default 0:
                          scheduled, 1 to 4 iterations ahead, from the decay of
                          each active residual towards its replacement or
                          stopping threshold, weighing the iterations that
                          states would run past it against the cost of a check
                          (2 under graph capture and in block COCG, 1 in
                          iobm_smatrix_bloch) */
  int32_t keep_direction; /* at a residual replacement: 0 = restart the search
                          direction (p = z; default), 1 = keep it (the
                          recurrence continues from the replaced residual; it
                          still restarts after a breakdown, a diverging
                          residual or a replacement that did not lower the true
                          residual).  Ignored with IOBM_PC_LATERAL_FFT, where
                          keeping it was measured to diverge */
  int32_t graph;       /* 1: the iterations between two convergence checks are
                          captured once into a HIP graph (on a stream of the
                          library, ordered after the caller's stream by events)
                          and replayed while the set of unconverged right-hand
                          sides stays the same; 0: launched one by one.  Same
                          kernels in the same order either way (bit-identical
                          results).  Ignored while the timing hook is on.
                          Default 0 */
  int32_t block;       /* 0: every state iterates on its own (per-state COCG
                          scalars); 1: block COCG per energy: the states of one
                          energy (at most 64) share one Krylov space, with the
                          s x s Grams P^T A P and R^T Z (FP64, matrix cores)
                          and s x s solves in place of the scalars.  Complex128
                          only (UNSUPPORTED with IOBM_C64_REFINED: the complex64
                          block recurrence diverges once the columns become
                          nearly dependent).  Default 0 */
  int32_t pad_;
} iobm_solve_opts;

/* Per (energy, incident channel) statistics (the paper's Table 2 counts
 * iterations).  A channel with G != 0 is solved as the cos and sin standing
 * waves of its +-G pair; its counts are the sums over those two solves. */
typedef struct {
  int32_t iters;        /* preconditioned COCG iterations */
  int32_t refinements;  /* FP64 true-residual evaluations (reliable updates) */
  int32_t status;       /* IOBM_OK or IOBM_E_NOT_CONVERGED / IOBM_E_BREAKDOWN */
  int32_t pad_;
  double rel_residual;  /* final ||b - A psi|| / ||b|| in FP64 */
  double flux_error;    /* T + R - 1 */
} iobm_solve_stat;

/* Fill opts with the defaults listed above. */
void iobm_default_opts(iobm_solve_opts* opts);

/* Create a context on the current HIP device.  hip_stream: hipStream_t or NULL.
 * The grid is copied.  Sizes: nf in 1..3, nx, ny >= max(2, nf), nz >= 2 nf,
 * finite h > 0.  Errors: INVALID_ARG (sizes, nf), UNSUPPORTED
 * (nx*ny > 4096, nz > 256, a lateral size with a prime factor > 31, or
 * (nf + 1) * nx*ny * 16 bytes beyond the device's LDS per workgroup: on
 * MI355X (160 KiB) nx*ny <= 4096, 3413 and 2560 for nf = 1, 2, 3),
 * DEVICE, OOM. */
iobm_status iobm_create(const iobm_grid* grid, void* hip_stream, iobm_ctx* out);

/* Set the local potential V(r) (Ha), float64 [nz][ny][nx], copied into the
 * context (Eq. (2): the diagonal of H(z_k)).  on_device: 0 = host pointer,
 * 1 = device pointer.  Errors: INVALID_ARG (NULL, non-finite value). */
iobm_status iobm_set_potential(iobm_ctx ctx, const double* V, int32_t on_device);

/* Set a separable (Kleinman-Bylander form) nonlocal term
 *     V_NL = sum_a B_a D_a h^3 B_a^T,  h^3 = hx*hy*hz,
 * added to H_T (the pseudopotential part of the Kohn-Sham Hamiltonian of
 * Sec. III/IV; synthetic here).  ncenters >= 0 (0 removes the term), rank in
 * 1..8; nsupport[a] = voxels of centre a; support_idx = concatenated flat
 * voxel ids (host, int64); beta = concatenated per-centre [rank][nsupport[a]]
 * float64 values (host); D = [ncenters][rank][rank] float64 (host), must be
 * symmetric so that A stays complex symmetric.  Data are copied.
 * Errors: INVALID_ARG (index out of range, non-symmetric D, non-finite). */
iobm_status iobm_set_nonlocal(iobm_ctx ctx, int32_t ncenters, int32_t rank,
                              const int32_t* nsupport, const int64_t* support_idx,
                              const double* beta, const double* D);

/* Open lateral channels at energy E (Eqs. (12)-(13), generalised to order
 * 2*nf): nopen = number of propagating modes.  Optional host outputs (may be
 * NULL, else sized by the caller to nx*ny): ids (ascending channel ids),
 * kz (propagating z wave number, 1/bohr, in (0, pi/hz)), v (group velocity,
 * bohr/a.u. time).  Errors: AT_THRESHOLD, INVALID_ARG. */
iobm_status iobm_channels(iobm_ctx ctx, double E, int32_t* nopen, int32_t* ids,
                          double* kz, double* v);

/* Self-energy of the right electrode in lateral-mode space (Eq. (15); an
 * nf x nf block per mode, plane index i <-> plane nz-nf+i), complex128
 * interleaved, host array [nx*ny][nf][nf].  The left electrode's block is
 * the same with the plane order reversed. */
iobm_status iobm_self_energy(iobm_ctx ctx, double E, double* sigma);

/* y = A(E) x for nrhs vectors: the FD stencil + (E - V) diagonal + nonlocal
 * term + FFT-applied electrode self-energies (Eqs. (6), (8), (14)-(16)).
 * x, y: device arrays [nrhs][nz][ny][nx] of complex128 (precision
 * IOBM_C128) or complex64 (IOBM_C64_REFINED); x and y must not overlap.
 * Asynchronous on the context stream. */
iobm_status iobm_apply(iobm_ctx ctx, double E, int32_t nrhs, const void* x, void* y,
                       int32_t precision);

/* z = P r for nrhs vectors with the preconditioner `precond` (IOBM_PC_*) at
 * energy E (only IOBM_PC_LATERAL_FFT depends on E), same layout rules as
 * iobm_apply.  rz: NULL, or host complex128 [nrhs] that receives the bilinear
 * form r^T z of each vector (no conjugation), from the same FP64-accumulated
 * partials that the solver's COCG step takes (for IOBM_PC_LATERAL_FFT they
 * come from the inverse plane FFT, in mode space).  Asynchronous when rz is
 * NULL; synchronises the stream otherwise. */
iobm_status iobm_precondition(iobm_ctx ctx, int32_t precond, double alpha, double E,
                              int32_t nrhs, const void* r, void* z, int32_t precision, double* rz);

/* iobm_precondition for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same operation, arguments, layouts, results and errors as
 * iobm_precondition for IOBM_PC_NONE, IOBM_PC_TRUNCATED_LAPLACIAN and
 * IOBM_PC_LATERAL_FFT (IOBM_PC_JACOBI returns INVALID_ARG here), and it
 * calls no hipMalloc, hipFree or other allocating routine.  Every device workspace it needs (the energy's mode table and
 * the plane-FFT scratch of IOBM_PC_LATERAL_FFT, the partial sums of r^T z)
 * lives in a static workspace of IOBM_STATIC_WORKSPACE_BYTES that the
 * library holds on every device it runs on until the process ends.  Needed:
 * IOBM_PC_LATERAL_FFT nrhs * nx*ny*nz * (16 bytes complex128, 8 complex64)
 * + 488 * nx*ny bytes; with rz, nrhs * (32 * slots + 16) bytes, slots = nz
 * (lateral-Fourier), ceil(nz / 16) (Eq. (17)) or up to 64 (none).  A request
 * beyond the workspace returns IOBM_E_UNSUPPORTED before any launch.
 * Every call on one device shares that device's workspace and leaves its
 * contents behind: calls that overlap on one GPU (several contexts, threads
 * or streams) race and must be serialised by the caller.  The context's
 * cached mode tables are not touched.  Synchronises the stream for
 * IOBM_PC_LATERAL_FFT (the threshold check of E) and when rz is requested;
 * otherwise asynchronous. */
#define IOBM_STATIC_WORKSPACE_BYTES (64ull << 20)
iobm_status iobm_precondition_noalloc(iobm_ctx ctx, int32_t precond, double alpha, double E,
                                      int32_t nrhs, const void* r, void* z, int32_t precision,
                                      double* rz);

/* Right-hand side of Eq. (6) for incident channels: b[c] for energy E and
 * channel ids[c] (must be open), device complex128 [n][nz][ny][nx], zero
 * outside the first (side 0) or last (side 1) nf planes. */
iobm_status iobm_rhs(iobm_ctx ctx, double E, int32_t n, const int32_t* ids, int32_t side,
                     void* b);

/* Solve Eq. (6) for every (energy, incident channel) pair and read out the
 * scattering amplitudes.
 *  nE energies E[e] (host); ninc[e] channel ids for energy e, concatenated in
 *  inc (host; ninc[e] = -1 means "every open channel at E[e]" and consumes no
 *  entries of inc).  nrhs = total number of pairs, in this order.
 *  psi: device [nrhs][nz][ny][nx] complex128, or NULL.
 *  t:   host, per energy [nopen(E)][ninc_e] complex128 (outgoing amplitudes of
 *       every open channel, concatenated over energies), or NULL.
 *  T, R: host [nrhs] float64, or NULL.  st: host [nrhs], or NULL.
 * Synchronises the stream.  Returns NOT_CONVERGED if any pair missed tol. */
iobm_status iobm_solve(iobm_ctx ctx, const iobm_solve_opts* opts, int32_t nE, const double* E,
                       const int32_t* ninc, const int32_t* inc, void* psi, double* t,
                       double* T, double* R, iobm_solve_stat* st);

/* Scattering matrix of each energy (the scattering condition, Eq. (7), with
 * incidence from both electrodes; the transmission block is the T matrix of
 * Sec. IV).  For energy e with n = nopen(E[e]) open channels (ascending ids,
 * as iobm_channels), S[e] is 2n x 2n, rows and columns ordered [left-lead
 * channels | right-lead channels]:
 *     S[b nu][a mu] = sqrt(v_nu / v_mu) * amplitude of the outgoing wave in
 *                     channel nu of lead b for a unit incident wave in
 *                     channel mu from lead a,
 * every amplitude (incident and outgoing) referred to the transition-region
 * plane next to its lead (plane 0 for the left lead, nz-1 for the right).
 * Flux conservation makes S unitary; with real V and kappa = 0 time
 * reversal gives S[b nu][a mu] = S[a -mu][b -nu], -mu being the channel of
 * the opposite lateral wave vector.  Runs every open channel from both
 * sides (2 sum_e n_e scattering states).
 *  S:  host complex128 interleaved, row-major, concatenated over energies
 *      (sum_e 4 n_e^2 entries).
 *  st: host [2 sum_e n_e] (left incidence first, then right), or NULL.
 * Synchronises the stream.  Returns NOT_CONVERGED if any state missed tol. */
iobm_status iobm_smatrix(iobm_ctx ctx, const iobm_solve_opts* opts, int32_t nE, const double* E, double* S,
                         iobm_solve_stat* st);

/* Lateral Bloch vector kappa = (kx, ky) (1/bohr): wave functions obey
 * psi(r + L_mu e_mu) = exp(i kappa_mu L_mu) psi(r) across the lateral cell
 * (Eq. (2)); the lateral waves are exp(i (G + kappa).r) (Eq. (16)) and every
 * lateral energy, Bloch root and self-energy is taken at G + kappa (Eqs.
 * (12)-(15)).  Channel ids are those of G, as for kappa = 0.
 *
 * Open channels at E and kappa: as iobm_channels. */
iobm_status iobm_channels_bloch(iobm_ctx ctx, double E, double kx, double ky, int32_t* nopen, int32_t* ids,
                                double* kz, double* v);

/* Scattering matrices at kappa and at -kappa, for each energy (Eq. (7) with
 * incidence from both electrodes, as iobm_smatrix, which is the case
 * kappa = 0).  With kappa != 0 the operator is not complex symmetric
 * (A(kappa)^T = A(-kappa)), so every state at kappa (channel mu) is solved
 * together with its time-reversal partner at -kappa (channel -mu, the
 * opposite lateral wave vector, same incident side) by biconjugate gradients
 * with the bilinear form; the pair shares its iteration.
 *  kx, ky: the Bloch vector (finite; any value, also 0 or the zone edge).
 *  S_plus, S_minus: host complex128 interleaved, concatenated over energies;
 *      energy e has n_e open channels (the same number at kappa and -kappa)
 *      and its matrix is 2n_e x 2n_e, ordered [left | right], channels in
 *      ascending ids of iobm_channels_bloch at kappa (S_plus) and at -kappa
 *      (S_minus), flux normalised and referred to the planes next to the
 *      leads as in iobm_smatrix.  Reciprocity gives
 *      S_plus[b nu][a mu] = S_minus[a -mu][b -nu].
 *  st: host [2 sum_e n_e] per pair (left incidence first), or NULL;
 *      flux_error is that of the state at kappa.
 *  opts: block must be 0 (UNSUPPORTED otherwise); precision, precond,
 *      alpha, tol, max_iter, check_every and inner_tol apply (IOBM_C64_REFINED:
 *      complex64 pair recurrences on a correction of the FP64 solution, the
 *      pair restarted from its FP64 true residual each time both recursive
 *      residuals have fallen by inner_tol); keep_direction and graph are
 *      ignored.
 * Errors: UNSUPPORTED with a nonlocal term set (iobm_set_nonlocal);
 * AT_THRESHOLD; NOT_CONVERGED / BREAKDOWN if a pair missed tol (the
 * matrices are still written).  Synchronises the stream. */
iobm_status iobm_smatrix_bloch(iobm_ctx ctx, const iobm_solve_opts* opts, double kx, double ky, int32_t nE,
                               const double* E, double* S_plus, double* S_minus, iobm_solve_stat* st);

/* Total transmission T_tot = sum over energies and every open incident
 * channel of T_mu, and its gradient with respect to the local potential,
 * dT_tot/dV(r), by one adjoint solve per channel with the same (complex
 * symmetric) operator.  The forward and adjoint states are solved as one
 * batch, so the context's workspaces hold twice the states that
 * iobm_solve would on the same energies.  T_total: host scalar; dT_dV:
 * device float64 [nz][ny][nx] (overwritten).  Synchronises the stream. */
iobm_status iobm_grad_transmission(iobm_ctx ctx, const iobm_solve_opts* opts, int32_t nE,
                                   const double* E, double* T_total, void* dT_dV);

/* Launch shapes of the volume kernels: a tuning knob, not part of the
 * method.  By default the first solve of a context in each precision times
 * the admissible stencil shapes and z-filter chunk lengths on its own batch
 * and keeps the fastest (the autotuner).  Shapes change the order in which
 * the FP64 partial sums of the COCG inner products are combined, so two
 * contexts tuned on their own may differ in the last bits (|Delta T| at the
 * solver tolerance).  Pinning the same shape in both makes them run the same
 * kernels in the same order: bit-identical results for identical input.
 * A zero field means "the default rule".
 *   stencil:           1 = 2.5D register-window stencil, 2 = cache-based stencil
 *   points_per_thread: 2.5D stencil, 1..4 (4 only for nf = 1); the block is
 *                      ceil(nx*ny / ppt) threads, which must fit the variant's
 *                      bound (1024, 1024, 768 and 640 threads)
 *   planes_per_block:  2.5D stencil, 8, 16, 32 or 64: the longest z chunk of a
 *                      block (small batches get shorter chunks, so that every
 *                      compute unit has blocks)
 *   zfilter_chunk:     lateral-Fourier preconditioner, 8, 16 or 32 planes per
 *                      chunk of the z recursion (at most 8 chunks)
 *   plane_fft:         1 = in-register plane FFT (square planes of 8, 12, 16,
 *                      24, 32 or 48 points), 2 = LDS Stockham plane FFT
 *   rz_pass:           lateral-Fourier preconditioner with the in-register
 *                      plane FFT: the pass that forms the r^T z partials,
 *                      1 = the z filter (each mode beside its negative in one
 *                      wavefront; used where its pair blocks fit the nz
 *                      partial slots of a state), 2 = the inverse plane FFT
 *                      (the autotuner times both and keeps the faster)
 * Shapes are kept per kernel arithmetic: IOBM_C64_REFINED selects the
 * complex64 kernels of the inner iteration, IOBM_C128 the complex128 ones
 * (including the FP64 residual refresh of a IOBM_C64_REFINED solve).
 * iobm_get_launch_shape returns the shape in effect for `precision` with
 * every field resolved.
 * iobm_set_launch_shape pins `shape` for that precision (the autotuner no
 * longer runs for it); shape = NULL unpins, and the next solve tunes again.
 * Errors: INVALID_ARG (field out of range), UNSUPPORTED (the shape does not
 * fit this grid). */
typedef struct {
  int32_t stencil;
  int32_t points_per_thread;
  int32_t planes_per_block;
  int32_t zfilter_chunk;
  int32_t plane_fft;
  int32_t rz_pass;
} iobm_launch_shape;
iobm_status iobm_get_launch_shape(iobm_ctx ctx, int32_t precision, iobm_launch_shape* shape);
iobm_status iobm_set_launch_shape(iobm_ctx ctx, int32_t precision, const iobm_launch_shape* shape);

/* Benchmark hook (not part of the method): time the launches of selected
 * kernel classes with HIP events recorded on the context stream around each
 * launch.  iobm_profile_begin clears the record and selects the classes
 * (bit mask of 1 << IOBM_K_*; 0 switches timing off).  iobm_profile_end
 * synchronises the stream and returns, for one class, the number of timed
 * launches, their summed duration (ms) and their summed algorithmic bytes:
 * per launch, every vector the launch must read or write, counted once
 * (shared tables such as V and the mode data not counted).  The record is
 * kept until the next iobm_profile_begin.  Classes of one kernel each,
 * except IOBM_K_PRECOND_FFT, which spans the three launches of the
 * lateral-Fourier preconditioner (algorithmic bytes: read r, write z). */
enum { IOBM_K_STENCIL = 1,      /* stencil in the iteration precision; with the
                                   fused direction update: read z, p_old, d,
                                   write p_new, y, d (d += alpha p_old; z only,
                                   p_new and y right after a restart); else
                                   read x, write y */
       IOBM_K_BOUNDARY = 2,     /* electrode term on the 2 nf face planes */
       IOBM_K_PRECOND_FFT = 3,  /* the whole lateral-Fourier preconditioner */
       IOBM_K_PRECOND_LAP = 4,  /* Eq. (17) preconditioner */
       IOBM_K_NONLOCAL = 5,     /* nonlocal projection on MFMA, complex64; its figure
                                   is algorithmic flops, 2 n_proj (2 n_rhs) n_support,
                                   not bytes */
       IOBM_K_DOT = 6,          /* bilinear / norm reductions */
       IOBM_K_UPDATE = 7,       /* r -= alpha q, |r|^2 partials */
       IOBM_K_STENCIL_C128 = 8, /* stencil in complex128 (FP64 residuals) */
       IOBM_K_FFT_PLANES = 9,   /* forward batched 2D plane FFT of the preconditioner */
       IOBM_K_ZFILTER = 10,     /* the z recursion of the preconditioner */
       IOBM_K_ACCUMULATE = 11,  /* x += d + alpha p, d = 0 (refinement) */
       IOBM_K_NONLOCAL_C128 = 12, /* as IOBM_K_NONLOCAL, complex128 (flops) */
       IOBM_K_FFT_PLANES_DOT = 13, /* inverse plane FFT with the r^T z partials */
       IOBM_K_FFT_PLANES_UPD = 14, /* forward plane FFT of q with the mode-space
                                   residual update R -= alpha FFT(q) */
       IOBM_K_PRECOND_JACOBI = 15,  /* Jacobi preconditioner: read r, write z */
       IOBM_K_BLOCK_GRAM = 16,      /* block COCG: s x s Grams of a group (MFMA f64) + their
                                       fixed-order sum; bytes: read both blocks once */
       IOBM_K_BLOCK_UPDATE = 17,    /* block COCG: Y (+/-)= X C or Y = Z + X C */
       IOBM_K_BLOCH_STENCIL = 18,   /* stencil with lateral bond phases (kappa != 0) */
       IOBM_K_BLOCH_VECTOR = 19 };  /* kappa != 0: pair inner products, updates, residuals, directions */
iobm_status iobm_profile_begin(iobm_ctx ctx, int32_t class_mask);
iobm_status iobm_profile_end(iobm_ctx ctx, int32_t kernel_class, int32_t* launches, double* total_ms,
                             double* alg_bytes);

iobm_status iobm_destroy(iobm_ctx ctx);
const char* iobm_status_str(iobm_status s);
const char* iobm_last_error(iobm_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* IOBM_H */
