// C ABI of libiobm: context management, validation, mode tables, and the
// batched preconditioned COCG driver with FP64 iterative refinement.
//
// Solver (Sec. II, last part, and Sec. III): the IOBM matrix is complex
// symmetric (A^T = A for real V, kappa = 0, symmetric Sigma and nonlocal
// term), so the conjugate-gradient iteration the paper uses is taken in its
// complex-orthogonal form (COCG: the bilinear form x^T y replaces x^H y).
// Every right-hand side of a batch carries its own energy and scalars.
//
// Lateral plane-wave incident channels exp(i G.r) with G != 0 have
// b^T b = 0 exactly (the lateral sum of exp(2 i G.r) vanishes), which breaks
// COCG down at its first step.  The driver therefore solves for the real
// lateral standing waves cos(G.r) and sin(G.r) of each +-G pair and combines
// psi_{+-G} = psi_cos +- i psi_sin (exact by linearity).
//
// Precision: IOBM_C128 runs COCG in complex128.  IOBM_C64_REFINED keeps the
// solution and the true residual r = b - A x in complex128 and solves the
// correction equation A d = r with complex64 COCG (FP64 inner products),
// x += d, until ||r|| <= tol ||b||.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

// Static device workspace of iobm_precondition_noalloc: a file-scope array
// that every GPU the library runs on holds until the process ends.  Its name
// is a host-side stand-in in host code, never a device address: iobm_create
// looks up this device's address once per device (hipGetSymbolAddress, with
// that device current) and host code uses only that address.
#define IOBM_STATIC_WS_BYTES (64ull << 20)
static __device__ __align__(256) unsigned char scratch[IOBM_STATIC_WS_BYTES];

// launchers from ops.hip
hipError_t launch_face_norm2(iobm_ctx c, const zd* b, int nact, const int* active, Partial* part);
template <typename T>
hipError_t launch_init_r(iobm_ctx c, const zd* b, cplx<T>* r, int nact, const int* active);
template <typename T>
hipError_t launch_dot(iobm_ctx c, const cplx<T>* a, const cplx<T>* b, int nact, const int* active, void* part);
template <typename T>
hipError_t launch_update_r(iobm_ctx c, cplx<T>* r, const cplx<T>* q, const zd* alpha, int nact, const int* active,
                           void* part);
enum { FIN_ALPHA = 0, FIN_BETA = 1, FIN_RESTART = 2, FIN_NORM = 3, FIN_KEEP = 4 };
hipError_t launch_finish2(iobm_ctx c, zd* rho, zd* alpha, zd* beta, double* rn2, int* flag, const Partial* pa,
                          int na, const Partial* pb, int nb, int mode, int nact, const int* active,
                          int* xset = nullptr, int* dlive = nullptr);
template <typename T>
hipError_t launch_residual(iobm_ctx c, const zd* b, cplx<T>* y, int nact, const int* active);
template <typename TD, typename TS>
hipError_t launch_convert(iobm_ctx c, const cplx<TS>* src, cplx<TD>* dst, int nact, const int* active);
template <typename T>
hipError_t launch_accumulate(iobm_ctx c, zd* x, const cplx<T>* d, const cplx<T>* p, const zd* alpha,
                             const int* xset, const int* dlive, int nact, const int* active, int nfirst, int ndead);
template <typename TR>
hipError_t launch_refresh(iobm_ctx c, const zd* x, const zd* b, zd* rface, cplx<TR>* r, int nrhs,
                          const double* E_rhs, const int* e_rhs, const ModeData* modes, const int* active,
                          Partial* part);
hipError_t launch_combine(iobm_ctx c, int nreq, const int* req_e, const int* req_mode, const int* req_c,
                          const int* req_s, const int* req_sgn, const ModeData* modes, const zd* amp_near,
                          const zd* amp_far, zd* t_out, zd* r_out, double* T, double* R);
template <typename TO>
hipError_t launch_combine_psi(iobm_ctx c, int nreq, const zd* x, cplx<TO>* psi, const int* req_c,
                              const int* req_s, const int* req_sgn);
// grad.hip
hipError_t launch_rhs_adjoint(iobm_ctx c, int nrhs, const int* e_rhs, const int* mode_rhs, const int* kind_rhs,
                              int side, const ModeData* modes, zd* b);
hipError_t launch_grad_D(iobm_ctx c, int nE, int nmax, const int* base, const int* chan, const zd* pcoef,
                         const zd* qcoef, const int* req_mode, const int* req_e, const ModeData* modes,
                         const zd* tamp, zd* D, const long long* dbase);
hipError_t launch_grad(iobm_ctx c, int nE, const int* base, const long long* dbase, const zd* D, const zd* u,
                       const zd* w, double* g);

// block.hip
template <typename T>
hipError_t launch_gram(iobm_ctx c, const cplx<T>* U, const cplx<T>* W, int ngroups, const int* cols,
                       const int* goff, const int* gsize, const int* gid, const int* poff, double* part, int nblk,
                       zd* G, int ncols);
hipError_t launch_small_solve(iobm_ctx c, int ngroups, const int* gsize, const int* gid, const zd* G, const zd* Y,
                              zd* Gw, zd* X, int* flag);
template <typename T, typename TY>
hipError_t launch_block_update(iobm_ctx c, cplx<TY>* Y, const cplx<T>* X, const cplx<T>* Z, const zd* C, int ngroups,
                               const int* cols, const int* goff, const int* gsize, const int* gid, int nchunk,
                               int mode, Partial* n2part, int ncols);

// bloch.hip
template <typename T>
hipError_t launch_bloch_apply_fused(iobm_ctx c, const BlochPhase& ph, const BlochFuse<T>& F, cplx<T>* y, int nrhs,
                                    const double* E_rhs, const int* e_rhs, const int* sgn, const int* active);
template <typename T>
hipError_t launch_bloch_laplacian(iobm_ctx c, const BlochPhase& ph, double alpha, const cplx<T>* r, cplx<T>* z,
                                  int nrhs, const int* sgn, const int* active);
template <typename T>
hipError_t launch_bloch_dot(iobm_ctx c, const cplx<T>* u, const cplx<T>* v, int npairs, const int* pairs,
                            Partial* part, int nblk);
hipError_t launch_bloch_scalars(iobm_ctx c, int mode, int npairs, const int* pairs, const Partial* pd, const Partial* pn,
                                int nblk, zd* rho, zd* alpha, zd* beta, double* rn2, int* flag);
template <typename T>
hipError_t launch_bloch_update(iobm_ctx c, cplx<T>* r, const cplx<T>* q, const zd* alpha, int nslots,
                               const int* active, Partial* pn, int nblk);
template <typename T>
hipError_t launch_bloch_settle(iobm_ctx c, zd* x, cplx<T>* d, const cplx<T>* p, const zd* alpha, int nslots,
                               const int* active, int nblk);

namespace {

struct Fail {
  iobm_status s;
};

const int kMaxDevices = 64;
std::mutex static_ws_mu;
void* static_ws_ptr[kMaxDevices] = {};

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                         \
      throw Fail{e_ == hipErrorOutOfMemory || e_ == hipErrorMemoryAllocation ? IOBM_E_OOM   \
                                                                              : IOBM_E_DEVICE}; \
    }                                                                                       \
  } while (0)

iobm_status fail(iobm_ctx ctx, iobm_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

// ------------------------------------------------------------- scratch pool
enum Slot {
  S_B, S_XHI, S_RHI, S_Y, S_R, S_Z, S_P, S_P2, S_Q, S_D, S_PF, S_PART, S_PARTA, S_PARTZ, S_PARTR, S_PARTN, S_SCAL,
  S_IDX, S_AMP,
  S_TR, S_KB, S_GRAD_D, S_BLK_PART, S_BLK_G, S_BLK_N2, NSLOT
};

void* workspace(iobm_ctx ctx, int slot, size_t bytes) {
  if ((int)ctx->pool.size() < NSLOT) ctx->pool.resize(NSLOT, {nullptr, 0});
  auto& e = ctx->pool[slot];
  if (e.second < bytes) {
    if (e.first) {
      (void)hipStreamSynchronize(ctx->stream);  // queued work may still use the old buffer
      (void)hipFree(e.first);
    }
    e.first = nullptr;
    e.second = 0;
    void* p = nullptr;
    hipError_t err = hipMalloc(&p, std::max<size_t>(bytes, 256));
    if (err != hipSuccess) {
      ctx->err = std::string("hipMalloc: ") + hipGetErrorString(err);
      throw Fail{IOBM_E_OOM};
    }
    e.first = p;
    e.second = std::max<size_t>(bytes, 256);
  }
  return e.first;
}

// Small index / scalar arrays go through a fixed device arena of 64 regions
// of 64 KB with a pinned host mirror.  An asynchronous copy reads the pinned
// mirror when it executes, and queued kernels read the device region when
// they run, so a region with an upload that the stream has not yet passed
// is never rewritten: the stream is synchronised first (region_pending).
const size_t kRegion = 64 * 1024;
const int kRegions = 64;

void stream_sync(iobm_ctx ctx) {
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    ctx->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
    throw Fail{IOBM_E_DEVICE};
  }
  for (int r = 0; r < kRegions; ++r) ctx->region_pending[r] = 0;
}

template <typename T>
T* upload(iobm_ctx ctx, int slot, const std::vector<T>& v, size_t offset_bytes = 0) {
  (void)slot;
  const size_t bytes = v.size() * sizeof(T);
  const size_t region = offset_bytes / 8192;  // offsets below are multiples of 8 KB
  if (region >= (size_t)kRegions - 1 || bytes > kRegion) {
    ctx->err = "index array too large (more than 8192 right-hand sides)";
    throw Fail{IOBM_E_UNSUPPORTED};
  }
  if (ctx->region_pending[region]) stream_sync(ctx);
  T* p = (T*)((char*)ctx->arena_d + region * kRegion);
  if (bytes) {
    memcpy((char*)ctx->arena_h + region * kRegion, v.data(), bytes);
    HIPCHK(hipMemcpyAsync(p, (char*)ctx->arena_h + region * kRegion, bytes, hipMemcpyHostToDevice,
                          ctx->stream));
    ctx->region_pending[region] = 1;
  }
  return p;
}

// Pinned host buffer for device-to-host read-backs of per-rhs scalars (a
// copy into pageable memory would be staged and serialised by the runtime).
void* pinned_readback(iobm_ctx ctx, size_t bytes) {
  if (ctx->rb_cap < bytes) {
    stream_sync(ctx);  // an earlier read-back may still target the old buffer
    if (ctx->rb_h) (void)hipHostFree(ctx->rb_h);
    ctx->rb_h = nullptr;
    ctx->rb_cap = 0;
    HIPCHK(hipHostMalloc(&ctx->rb_h, bytes, hipHostMallocDefault));
    ctx->rb_cap = bytes;
  }
  return ctx->rb_h;
}

FFTPlan1D make_plan1d(int n) {
  FFTPlan1D p;
  p.n = n;
  p.nstages = 0;
  int m = n;
  while (m % 4 == 0) { p.radix[p.nstages++] = 4; m /= 4; }
  while (m % 2 == 0) { p.radix[p.nstages++] = 2; m /= 2; }
  for (int f = 3; m > 1; f += 2)
    while (m % f == 0) { p.radix[p.nstages++] = f; m /= f; }
  return p;
}

bool plan_ok(const FFTPlan1D& p) {
  if (p.nstages > IOBM_FFT_MAXSTAGES) return false;
  for (int s = 0; s < p.nstages; ++s)
    if (p.radix[s] > 31) return false;
  return true;
}

// --------------------------------------------------------------- modes
// Ensure the device mode table holds exactly the energies `E` (in order),
// entry e at the lateral Bloch vector given by K[2e], K[2e+1] (phases per
// lattice step; K empty: kappa = 0 throughout).  Only the mode flags come
// back to the host; the full records are copied on demand (host_modes) by
// the calls that report them.
void ensure_modes(iobm_ctx ctx, const std::vector<double>& E, bool force = false,
                  const std::vector<double>& K = std::vector<double>()) {
  if (!force && E == ctx->modeE && K == ctx->modeK && ctx->modes_d) return;
  const size_t n = (size_t)E.size() * ctx->g.nxy;
  if (ctx->modes_cap < n) {
    if (ctx->modes_d) (void)hipFree(ctx->modes_d);
    ctx->modes_d = nullptr;
    ctx->modes_cap = 0;
    HIPCHK(hipMalloc(&ctx->modes_d, n * sizeof(ModeData)));
    ctx->modes_cap = n;
  }
  const size_t ns = n * ctx->g.nf * ctx->g.nf;
  if (ctx->sig_cap < ns) {
    if (ctx->sig_d) (void)hipFree(ctx->sig_d);
    if (ctx->sig_f) (void)hipFree(ctx->sig_f);
    if (ctx->mode_flags_d) (void)hipFree(ctx->mode_flags_d);
    if (ctx->sdiag_d) (void)hipFree(ctx->sdiag_d);
    ctx->sig_d = nullptr;
    ctx->sig_f = nullptr;
    ctx->mode_flags_d = nullptr;
    ctx->sdiag_d = nullptr;
    ctx->sig_cap = 0;
    HIPCHK(hipMalloc(&ctx->sig_d, ns * sizeof(zd)));
    HIPCHK(hipMalloc(&ctx->sig_f, ns * sizeof(zf)));
    HIPCHK(hipMalloc(&ctx->mode_flags_d, n * sizeof(int)));
    HIPCHK(hipMalloc(&ctx->sdiag_d, (size_t)E.size() * ctx->g.nxy * ctx->g.nf * sizeof(zd)));
    ctx->sig_cap = ns;
  }
  ctx->modeE.clear();
  ctx->modeK.clear();
  ctx->modes_h_valid = false;
  double* Ed = upload(ctx, S_IDX, E);
  double* Kd = K.empty() ? nullptr : upload(ctx, S_IDX, K, 64 * 1024);
  HIPCHK(launch_modes(ctx, Ed, (int)E.size(), ctx->modes_d, Kd));
  HIPCHK(launch_sigma_tables(ctx, (int)E.size(), ctx->modes_d, ctx->sig_d, ctx->sig_f, ctx->mode_flags_d));
  HIPCHK(launch_sigma_diag(ctx, (int)E.size()));
  int* fh = (int*)pinned_readback(ctx, n * sizeof(int));
  HIPCHK(hipMemcpyAsync(fh, ctx->mode_flags_d, n * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  stream_sync(ctx);
  ctx->mode_flags_h.assign(fh, fh + n);
  for (size_t e = 0; e < E.size(); ++e)
    for (int m = 0; m < ctx->g.nxy; ++m) {
      const int fl = ctx->mode_flags_h[e * ctx->g.nxy + m];
      if (fl & MODE_THRESHOLD) {
        char buf[160];
        snprintf(buf, sizeof buf, "energy %.12g is at the threshold of lateral channel %d", E[e], m);
        ctx->err = buf;
        throw Fail{IOBM_E_AT_THRESHOLD};
      }
      if (fl & MODE_FAIL) {
        char buf[160];
        snprintf(buf, sizeof buf, "mode setup failed at energy %.12g, channel %d", E[e], m);
        ctx->err = buf;
        throw Fail{IOBM_E_DEVICE};
      }
    }
  ctx->modeE = E;
  ctx->modeK = K;
}

// The full mode records of the current table on the host.
const ModeData* host_modes(iobm_ctx ctx) {
  if (!ctx->modes_h_valid) {
    const size_t n = ctx->modeE.size() * (size_t)ctx->g.nxy;
    ctx->modes_h.resize(n);
    HIPCHK(hipMemcpyAsync(ctx->modes_h.data(), ctx->modes_d, n * sizeof(ModeData), hipMemcpyDeviceToHost,
                          ctx->stream));
    stream_sync(ctx);
    ctx->modes_h_valid = true;
  }
  return ctx->modes_h.data();
}

int neg_mode(const GridDev& g, int m) {
  int ix = m % g.nx, iy = m / g.nx;
  return ((g.ny - iy) % g.ny) * g.nx + (g.nx - ix) % g.nx;
}

// ------------------------------------------------------------ the solver
struct Batch {
  int n = 0;                 // right-hand sides
  std::vector<int> e;        // energy index per rhs
  std::vector<double> E;     // energy per rhs
  std::vector<int> mode;     // lateral channel id (canonical member of the +-G pair)
  std::vector<int> kind;     // 1 cos, 2 sin
};

struct Request {
  std::vector<int> e, mode, c, s, sgn;
};

struct SolveOut {
  std::vector<int> iters, refin, status;
  std::vector<double> rel;
};

// Executable graph of one check's iterations, valid for one active list
// (count and device pointer) and one parity of the direction buffers.
struct CheckGraph {
  hipGraphExec_t exec = nullptr;
  int nact = -1;
  const int* act = nullptr;
  const void* pold = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    nact = -1;
  }
  ~CheckGraph() { reset(); }
};

// Batched preconditioned COCG with FP64 residual replacement (mixed precision).
//
// The Krylov recurrences run in type T (complex64 or complex128) on the
// correction d of the FP64 solution x: q = A p, alpha = rho / p^T q,
// d += alpha p, r -= alpha q, z = P r, beta = (r^T z) / rho, p = z + beta p,
// with every inner product accumulated in FP64.  The step d += alpha p is
// deferred to the next operator pass, which reads p anyway (alpha then
// holds the pending factor).  When the recursively updated residual of a
// right-hand side has fallen by the factor `delta` (opts.inner_tol) since
// its last update, or below the target, the correction is folded into x in
// FP64 (x += d + alpha p, d = 0), the true residual r = b - A x is formed
// with the complex128 operator and the iterated residual is replaced by it
// (a reliable update in the sense of van der Vorst and Ye).  The search
// direction then restarts (p = z), or, with opts.keep_direction, is kept
// across the replacement (beta from the replaced residual, p = z + beta p)
// unless the state broke down (vanishing rho or p^T q), diverged, or its true
// residual did not improve.  A right-hand side is done when its true
// residual is <= tol ||b||.
template <typename T>
void solve_rhs_batch(iobm_ctx ctx, const iobm_solve_opts& o, const Batch& B, const zd* b, zd* x, SolveOut& out) {
  const int nb = B.n;
  const long long vol = ctx->g.npts;
  out.iters.assign(nb, 0);
  out.refin.assign(nb, 0);
  out.status.assign(nb, IOBM_OK);
  out.rel.assign(nb, 0.0);
  if (nb == 0) return;
  const size_t vb = (size_t)nb * vol * sizeof(cplx<T>);
  int* e_d = upload(ctx, S_IDX, B.e, 0);
  double* E_d = upload(ctx, S_IDX, B.E, 16 * 1024);
  std::vector<int> all(nb);
  for (int i = 0; i < nb; ++i) all[i] = i;
  int* all_d = upload(ctx, S_IDX, all, 32 * 1024);
  zd* rhi = (zd*)workspace(ctx, S_RHI, (size_t)nb * vol * sizeof(zd));
  cplx<T>* d = (cplx<T>*)workspace(ctx, S_D, vb);
  cplx<T>* r = (cplx<T>*)workspace(ctx, S_R, vb);
  cplx<T>* pa = (cplx<T>*)workspace(ctx, S_P, vb);   // direction, two buffers used in turn
  cplx<T>* pb = (cplx<T>*)workspace(ctx, S_P2, vb);
  cplx<T>* q = (cplx<T>*)workspace(ctx, S_Q, vb);
  cplx<T>* z = o.precond == IOBM_PC_NONE ? r : (cplx<T>*)workspace(ctx, S_Z, vb);
  cplx<T>* pf = o.precond == IOBM_PC_LATERAL_FFT ? (cplx<T>*)workspace(ctx, S_PF, vb) : nullptr;
  const int nblk = dot_blocks(ctx);
  const int nz_slots = precond_slots(ctx, o.precond);
  Partial* part = (Partial*)workspace(ctx, S_PART, (size_t)nb * nblk * sizeof(Partial));
  Partial* part_pq = (Partial*)workspace(ctx, S_PARTA, (size_t)nb * PQ_SLOTS * sizeof(Partial));
  Partial* part_rz = o.precond == IOBM_PC_NONE
                         ? part
                         : (Partial*)workspace(ctx, S_PARTZ, (size_t)nb * nz_slots * sizeof(Partial));
  Partial* part_rn = (Partial*)workspace(ctx, S_PARTR, (size_t)nb * PQ_SLOTS * sizeof(Partial));
  // with the lateral-Fourier preconditioner on square planes, the update runs
  // inside its forward transform, which writes the |r|^2 partials per plane:
  // between replacements the iterated residual lives only in lateral mode
  // space (R = FFT(r) in pf, R -= alpha FFT(q)); the real-space r is formed
  // only by a replacement, whose preconditioner pass transforms it into pf
  const bool fuse_upd = o.precond == IOBM_PC_LATERAL_FFT && fft_reg_available<T>(ctx);
  Partial* part_n2 = fuse_upd ? (Partial*)workspace(ctx, S_PARTN, (size_t)nb * ctx->g.nz * sizeof(Partial)) : part;
  const int n2_slots = fuse_upd ? ctx->g.nz : nblk;
  // per-rhs scalars; |r|^2 and the breakdown flags are adjacent so that one
  // copy brings both to the host at a convergence check
  const size_t nb8 = ((size_t)nb + 1) & ~(size_t)1;
  char* sc = (char*)workspace(ctx, S_SCAL, (size_t)nb * 3 * sizeof(zd) + nb8 * (2 * sizeof(double) + 3 * sizeof(int)) + 64);
  zd* rho = (zd*)sc;
  zd* alpha = rho + nb;
  zd* beta = alpha + nb;
  double* rn2 = (double*)(beta + nb);
  int* flag = (int*)(rn2 + nb);
  double* tn2 = (double*)(flag + nb8);
  int* xset = (int*)(tn2 + nb8);  // 1 once a refinement has written x (x is not cleared up front)
  int* dlive = xset + nb8;        // 1 while d holds steps not yet folded into x
  const size_t check_bytes = (size_t)nb * sizeof(double) + (size_t)nb * sizeof(int);
  char* rbh = (char*)pinned_readback(ctx, check_bytes + nb8 * sizeof(int) + (size_t)nb * sizeof(double) + 64);
  const double* rn2_h = (const double*)rbh;
  const int* flag_h = (const int*)(rbh + (size_t)nb * sizeof(double));
  double* tn2_pin = (double*)(rbh + (size_t)nb * sizeof(double) + nb8 * sizeof(int));
  if (ctx->kb.ncen > 0) (void)kb_scratch(ctx, kb_proj_bytes(ctx, nb));
  const ModeData* modes = ctx->modes_d;
  const bool lowp = sizeof(T) == sizeof(float);
  const double tol2 = o.tol * o.tol;
  const double delta2 = lowp ? o.inner_tol * o.inner_tol : 0.0;
  // iterations per host check: fixed, or (check_every = 0, launched path)
  // scheduled from the observed decay of each active residual, between 1
  // and kMaxCheck (below)
  const bool graphs = o.graph != 0 && ctx->prof_mask == 0;
  const bool adapt = o.check_every == 0 && !graphs;
  constexpr int kMaxCheck = 4;
  constexpr double kCheckSeconds = 1e-4;          // a host check's round trip (measured: 50-120 us)
  constexpr double kStreamBytesPerSecond = 5e12;  // what the iteration's kernels stream (measured: 4.6-5.7 TB/s)
  int check = o.check_every > 0 ? o.check_every : (adapt ? 1 : 2);
  // keeping the direction across replacements diverged with the
  // lateral-Fourier preconditioner (measured): it always restarts there
  const bool keep_dir = o.keep_direction != 0 && o.precond != IOBM_PC_LATERAL_FFT;

  // z = P r for the listed rhs, with the partials of r^T z in part_rz (for
  // P = I they come from a separate reduction)
  auto precond = [&](int nact, const int* ad) {
    if (o.precond == IOBM_PC_TRUNCATED_LAPLACIAN)
      HIPCHK(launch_precond_laplacian<T>(ctx, o.alpha, r, z, nact, ad, part_rz));
    else if (o.precond == IOBM_PC_LATERAL_FFT)
      HIPCHK(launch_precond_fft<T>(ctx, r, z, pf, nact, e_d, modes, ad, part_rz));
    else if (o.precond == IOBM_PC_JACOBI)
      HIPCHK(launch_precond_jacobi<T>(ctx, r, z, nact, e_d, E_d, ad, part_rz));
    else
      HIPCHK(launch_dot<T>(ctx, r, r, nact, ad, part_rz));
  };
  std::vector<int> since(nb, 0);  // steps since the last replacement, per rhs (d holds data from 2 on)
  std::vector<char> kept(nb, 0);  // the last replacement kept the direction (p_old is read at its first step)
  std::vector<char> badv(nb, 0);  // breakdown or divergence seen at the last check
  cplx<T>* pold = pa;  // the direction of the last step (its update pending)
  cplx<T>* pnew = pb;
  // Refinement of the listed rhs: x += d + alpha p, d = 0, r = b - A x in FP64 (stored
  // in the iteration precision; the FP64 face planes pass through r_hi), and
  // |r|^2 -> host.  With a nonlocal term the residual is formed in full in
  // r_hi first, since its back-projection comes after the stencil.
  std::vector<double> tn2_h(nb), bn2(nb);
  auto read_tn2 = [&](std::vector<double>& dst) {
    HIPCHK(hipMemcpyAsync(tn2_pin, tn2, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    memcpy(dst.data(), tn2_pin, nb * sizeof(double));
  };
  auto refresh = [&](const std::vector<int>& lst, int region) {
    int* ld = upload(ctx, S_IDX, lst, (size_t)region * 8192);
    const int n = (int)lst.size();
    int nfirst = 0, ndead = 0;  // x not read (first refinement), d not read (no step since the last)
    for (int i : lst) { nfirst += out.refin[i] == 0; ndead += since[i] < 2; }
    HIPCHK(launch_accumulate<T>(ctx, x, d, pold, alpha, xset, dlive, n, ld, nfirst, ndead));
    if (ctx->kb.ncen == 0) {
      HIPCHK(launch_refresh<T>(ctx, x, b, rhi, r, n, E_d, e_d, modes, ld, part_rn));
      HIPCHK(launch_finish2(ctx, rho, alpha, beta, tn2, flag, part_rn, PQ_SLOTS, nullptr, 0, FIN_NORM, n, ld,
                            xset, dlive));
    } else {
      HIPCHK(launch_apply<double>(ctx, x, rhi, n, E_d, e_d, modes, ld));
      HIPCHK(launch_residual<double>(ctx, b, rhi, n, ld));
      HIPCHK(launch_dot<double>(ctx, rhi, rhi, n, ld, part));
      HIPCHK(launch_finish2(ctx, rho, alpha, beta, tn2, flag, part, nblk, nullptr, 0, FIN_NORM, n, ld, xset,
                            dlive));
      HIPCHK((launch_convert<T, double>(ctx, rhi, r, n, ld)));
    }
    read_tn2(tn2_h);
  };

  // start: x = 0 (written by the first refinement), d = 0, r = b, z = P r,
  // rho = r^T z, beta = 0
  HIPCHK(hipMemsetAsync(xset, 0, 2 * nb8 * sizeof(int), ctx->stream));  // xset and dlive
  HIPCHK(hipMemsetAsync(flag, 0, nb * sizeof(int), ctx->stream));
  HIPCHK(hipMemsetAsync(part_pq, 0, (size_t)nb * PQ_SLOTS * sizeof(Partial), ctx->stream));
  HIPCHK(hipMemsetAsync(part_rn, 0, (size_t)nb * PQ_SLOTS * sizeof(Partial), ctx->stream));
  // b vanishes between the 2 nf face planes (the solver's right-hand sides
  // are read there only)
  HIPCHK(launch_face_norm2(ctx, b, nb, all_d, part));
  HIPCHK(launch_finish2(ctx, rho, alpha, beta, tn2, flag, part, 1, nullptr, 0, FIN_NORM, nb, all_d));
  read_tn2(bn2);
  std::vector<int> act, zero;
  for (int i = 0; i < nb; ++i)
    (bn2[i] > 0 ? act : zero).push_back(i);
  // x = 0 for b = 0; every other rhs gets x from its first refinement
  if (!zero.empty()) HIPCHK((launch_convert<double, double>(ctx, nullptr, x, (int)zero.size(),
                                                             upload(ctx, S_IDX, zero, 48 * 1024))));
  std::vector<double> maxr2(nb), best(nb), last(nb);
  std::vector<int> stall(nb, 0);
  for (int i = 0; i < nb; ++i) maxr2[i] = best[i] = last[i] = bn2[i];
  tn2_h = bn2;
  // check schedule: |r|^2 at the last observation (a check, or the true
  // residual of a refresh), the iterations since, and the per-iteration
  // decay log(|r|^2) of the last observed stretch (0: none yet)
  std::vector<double> obs_r2(bn2), decay(nb, 0.0);
  std::vector<int> obs_it(nb, 0);
  if (act.empty()) return;
  int nact = (int)act.size();
  int* act_d = upload(ctx, S_IDX, act, 64 * 1024);
  HIPCHK(launch_init_r<T>(ctx, b, r, nact, act_d));
  if (!ctx->tuned[prec_index<T>()]) {
    // the shapes are timed on the fused operator with p_old = 0 and a
    // nonzero beta (0x3F bytes: 4.8e-4), so that every stream is read
    HIPCHK(hipMemsetAsync(pa, 0, vb, ctx->stream));
    HIPCHK(hipMemsetAsync(beta, 0x3F, nb * sizeof(zd), ctx->stream));
    HIPCHK(hipMemsetAsync(alpha, 0x3F, nb * sizeof(zd), ctx->stream));  // d += alpha * 0 leaves d = 0
    ApplyFuse<T> TF{r, pa, beta, pb, part_pq, alpha, d, dlive};
    autotune<T>(ctx, r, q, pf, nact, E_d, e_d, modes, act_d, &TF,
                o.precond == IOBM_PC_LATERAL_FFT ? part_rz : nullptr);
    HIPCHK(hipMemsetAsync(part_pq, 0, (size_t)nb * PQ_SLOTS * sizeof(Partial), ctx->stream));
  }
  precond(nact, act_d);
  HIPCHK(launch_finish2(ctx, rho, alpha, beta, rn2, flag, part_rz, nz_slots, nullptr, 0, FIN_RESTART, nact, act_d));

  // One iteration is three passes over the batch:
  //   operator:  p_new = z + beta p_old, q = A p_new, partials of p_new^T q
  //   update:    d += alpha p_new, r -= alpha q, partials of |r|^2 (and r^T r)
  //              (fused: inside the preconditioner's forward transform, on
  //              R = FFT(r) from FFT(q))
  //   precond:   z = P r, partials of r^T z
  // with the scalar steps (alpha; beta, rho, |r|^2) in between.
  // one check's iterations, launched one by one or captured into a graph
  CheckGraph cg;
  auto enqueue_check = [&]() {
    for (int k = 0; k < check; ++k) {
      int nfresh = 0, nfirstd = 0, nkept = 0;  // byte count only: steps since the replacement 0 and 1
      for (int i : act) {
        nfresh += since[i] + k == 0 && !kept[i];
        nkept += since[i] + k == 0 && kept[i];
        nfirstd += since[i] + k == 1;
      }
      ApplyFuse<T> F{z, pold, beta, pnew, part_pq, alpha, d, dlive, nfresh, nfirstd, nkept};
      HIPCHK(launch_apply<T>(ctx, nullptr, q, nact, E_d, e_d, modes, act_d, &F));
      HIPCHK(launch_finish2(ctx, rho, alpha, beta, rn2, flag, part_pq, PQ_SLOTS, nullptr, 0, FIN_ALPHA, nact, act_d,
                            nullptr, dlive));
      if (fuse_upd) {
        FftUpd<T> U;
        U.q = q; U.alpha = alpha; U.n2part = part_n2;
        HIPCHK(launch_precond_fft<T>(ctx, r, z, pf, nact, e_d, modes, act_d, part_rz, &U));
      } else {
        HIPCHK(launch_update_r<T>(ctx, r, q, alpha, nact, act_d, part));
        if (o.precond != IOBM_PC_NONE) precond(nact, act_d);  // P = I: r^T r came with the update
      }
      HIPCHK(launch_finish2(ctx, rho, alpha, beta, rn2, flag, part_rz, nz_slots, part_n2, n2_slots, FIN_BETA, nact,
                            act_d));
      std::swap(pold, pnew);
    }
  };
  auto run_check = [&]() {
    if (!graphs) {
      enqueue_check();
      return;
    }
    if (!ctx->cap_stream) {
      HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      for (hipEvent_t& ev : ctx->cap_ev) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    if (!cg.exec || cg.nact != nact || cg.act != act_d || cg.pold != (const void*)pold) {
      cg.reset();
      const void* p0 = pold;
      hipStream_t caller = ctx->stream;
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
      ctx->stream = ctx->cap_stream;  // every launcher enqueues on ctx->stream
      try {
        enqueue_check();
      } catch (Fail&) {
        ctx->stream = caller;
        (void)hipStreamEndCapture(ctx->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      ctx->stream = caller;
      HIPCHK(hipStreamEndCapture(ctx->cap_stream, &graph));
      const hipError_t ie = hipGraphInstantiate(&cg.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(ie);
      cg.nact = nact;
      cg.act = act_d;
      cg.pold = p0;
      if (check % 2) std::swap(pold, pnew);  // capture swapped them on the host: back to the launch state
    }
    HIPCHK(hipEventRecord(ctx->cap_ev[0], ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->cap_stream, ctx->cap_ev[0], 0));
    HIPCHK(hipGraphLaunch(cg.exec, ctx->cap_stream));
    HIPCHK(hipEventRecord(ctx->cap_ev[1], ctx->cap_stream));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->cap_ev[1], 0));
    if (check % 2) std::swap(pold, pnew);
  };
  while (nact > 0) {
    run_check();
    for (int i : act) since[i] += check;
    HIPCHK(hipMemcpyAsync(rbh, rn2, check_bytes, hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    // which rhs fold their correction into x and refresh the residual
    std::vector<int> upd;
    for (int i : act) {
      out.iters[i] += check;
      const double r2 = rn2_h[i];
      obs_it[i] += check;
      if (r2 > 0 && obs_r2[i] > 0 && r2 == r2) decay[i] = log(r2 / obs_r2[i]) / obs_it[i];
      obs_r2[i] = r2;
      obs_it[i] = 0;
      const bool bad = flag_h[i] || !(r2 == r2) || r2 > 1e4 * maxr2[i];  // breakdown or divergence
      badv[i] = bad;
      if (bad || r2 <= 0.25 * tol2 * bn2[i] || r2 <= delta2 * maxr2[i] || out.iters[i] >= o.max_iter)
        upd.push_back(i);
      else maxr2[i] = std::max(maxr2[i], r2);
    }
    if (!upd.empty()) {
      refresh(upd, 7);
      std::vector<int> rst, keep;  // updated rhs that go on iterating: from a restart / with the old direction
      for (int i : upd) {
        out.refin[i] += 1;
        const double t2 = tn2_h[i];
        if (t2 <= tol2 * bn2[i]) continue;  // converged
        if (out.iters[i] >= o.max_iter) { out.status[i] = IOBM_E_NOT_CONVERGED; continue; }
        const bool improved = t2 < best[i];
        if (t2 < 0.25 * best[i]) { best[i] = t2; stall[i] = 0; }
        else if (++stall[i] >= 6) {
          out.status[i] = flag_h[i] ? IOBM_E_BREAKDOWN : IOBM_E_NOT_CONVERGED;
          continue;
        }
        (keep_dir && !badv[i] && improved && since[i] > 0 ? keep : rst).push_back(i);
        maxr2[i] = t2;
      }
      std::vector<char> gone(nb, 0);
      for (int i : upd) gone[i] = 1;
      for (int i : rst) gone[i] = 0;
      for (int i : keep) gone[i] = 0;
      std::vector<int> lists(rst);  // one upload: [restarted rhs | kept rhs | new active list]
      lists.insert(lists.end(), keep.begin(), keep.end());
      for (int i : act)
        if (!gone[i]) lists.push_back(i);
      const int nr = (int)rst.size(), nk = (int)keep.size(), nc = nr + nk;
      int* ld = upload(ctx, S_IDX, lists, 64 * 1024);
      if (nc > 0) {
        // z = P r of the replaced residual, rho = r^T z; a restart sets beta = 0
        // (p_new = z next), a kept direction beta = rho' / rho (p_new = z + beta p)
        precond(nc, ld);
        if (nr) HIPCHK(launch_finish2(ctx, rho, alpha, beta, rn2, flag, part_rz, nz_slots, nullptr, 0, FIN_RESTART, nr, ld));
        if (nk) HIPCHK(launch_finish2(ctx, rho, alpha, beta, rn2, flag, part_rz, nz_slots, nullptr, 0, FIN_KEEP, nk, ld + nr));
      }
      act.assign(lists.begin() + nc, lists.end());
      nact = (int)act.size();
      act_d = ld + nc;  // the old list's region was rewritten
      for (int i : rst) { since[i] = 0; kept[i] = 0; }
      for (int i : keep) { since[i] = 0; kept[i] = 1; }
      for (int i : upd) obs_r2[i] = tn2_h[i];  // the true residual restarts the observation
    }
    if (adapt && nact > 0) {
      // Each active residual is predicted to reach its replacement or
      // stopping threshold after n_i more iterations (1 while it has no
      // observed decay yet, never while it grows).  A check after c
      // iterations costs a host round trip, s iterations' worth of the
      // batch's streaming; a rhs that passes its threshold before the check
      // runs c - n_i iterations that only its own share of the batch pays.
      // c in 1..kMaxCheck maximises the useful iterations per unit time,
      // (c - W(c)) / (c + s) with W(c) = mean over rhs of max(0, c - n_i).
      std::vector<int> hist(kMaxCheck + 1, 0);  // rhs with n_i = 1 .. kMaxCheck (and beyond)
      for (int i : act) {
        const double target = std::max(0.25 * tol2 * bn2[i], delta2 * maxr2[i]);
        int n = kMaxCheck;
        if (decay[i] == 0.0 || (decay[i] < 0.0 && obs_r2[i] <= target)) n = 1;
        else if (decay[i] < 0.0) n = (int)std::min<double>(kMaxCheck, ceil(log(target / obs_r2[i]) / decay[i]));
        hist[std::max(1, std::min(kMaxCheck, n))]++;
      }
      const double it_bytes = (lowp ? 112.0 : 224.0) * nact * (double)vol;  // one iteration's vector streams
      const double s_rel = kCheckSeconds / (it_bytes / kStreamBytesPerSecond);
      double best_rate = -1;
      for (int c = 1; c <= kMaxCheck; ++c) {
        double waste = 0;
        for (int n = 1; n < c; ++n) waste += (double)hist[n] * (c - n);
        const double rate = (c - waste / nact) / (c + s_rel);
        if (rate > best_rate) { best_rate = rate; check = c; }
      }
    }
  }
  for (int i = 0; i < nb; ++i) {
    out.rel[i] = bn2[i] > 0 ? sqrt(tn2_h[i] / bn2[i]) : 0.0;
    if (out.status[i] == IOBM_OK && bn2[i] > 0 && tn2_h[i] > tol2 * bn2[i]) out.status[i] = IOBM_E_NOT_CONVERGED;
  }
}

// Block COCG per energy (opts.block = 1).  The states of one energy form a
// group of s <= 64 columns that share the Krylov space: with R, Z, P, Q the
// blocks of the group's residuals, preconditioned residuals, directions and
// operator images,
//   alpha = (P^T Q)^-1 (R^T Z),  D += P alpha,  R -= Q alpha,  Z = M R,
//   beta = (R^T Z)_old^-1 (R^T Z)_new,  P = Z + P beta,
// with the s x s Grams accumulated in FP64 on the matrix cores and solved
// in FP64.  The recurrences run in complex128 on the correction D of the
// solution x (the driver is written for either iteration precision, but
// solve_batch admits complex128 only).  A group is refreshed (x += D, the
// true residual r = b - A x, converged columns leave, the recursion
// restarts with P = Z) when the iterated residuals of all its columns have
// reached the target, or a column's has fallen by opts.inner_tol
// (complex64) or diverged, or a Gram solve broke down (the block has become
// rank deficient).  Columns that reach the target early stay in the block
// until the group is refreshed: a refresh restarts the block Krylov space of
// every column of the group, and restarts at every converged column cost
// far more than the extra iterations (measured in a NumPy model of this
// driver: 135x the iterations of the plain recurrence on a Helmholtz test
// problem).  A group whose Gram solve broke down is split into single
// columns after its refresh; they keep their progress and continue as plain
// COCG.
template <typename T>
void solve_block_batch(iobm_ctx ctx, const iobm_solve_opts& o, const Batch& B, const zd* b, zd* x, SolveOut& out) {
  const int nb = B.n;
  const long long vol = ctx->g.npts;
  out.iters.assign(nb, 0);
  out.refin.assign(nb, 0);
  out.status.assign(nb, IOBM_OK);
  out.rel.assign(nb, 0.0);
  if (nb == 0) return;
  // groups: the consecutive states of one energy
  std::vector<int> gfirst, gsz;
  for (int i = 0; i < nb; ++i) {
    if (i == 0 || B.e[i] != B.e[i - 1]) {
      gfirst.push_back(i);
      gsz.push_back(0);
    }
    gsz.back()++;
  }
  const int ng = (int)gfirst.size();
  for (int g = 0; g < ng; ++g)
    if (gsz[g] > 64) {
      ctx->err = "block COCG takes at most 64 states per energy";
      throw Fail{IOBM_E_UNSUPPORTED};
    }
  const size_t vb = (size_t)nb * vol * sizeof(cplx<T>);
  int* e_d = upload(ctx, S_IDX, B.e, 0);
  double* E_d = upload(ctx, S_IDX, B.E, 16 * 1024);
  std::vector<int> all(nb);
  for (int i = 0; i < nb; ++i) all[i] = i;
  int* all_d = upload(ctx, S_IDX, all, 32 * 1024);
  zd* rhi = (zd*)workspace(ctx, S_RHI, (size_t)nb * vol * sizeof(zd));
  cplx<T>* d = (cplx<T>*)workspace(ctx, S_D, vb);
  cplx<T>* r = (cplx<T>*)workspace(ctx, S_R, vb);
  cplx<T>* pa = (cplx<T>*)workspace(ctx, S_P, vb);
  cplx<T>* pb = (cplx<T>*)workspace(ctx, S_P2, vb);
  cplx<T>* q = (cplx<T>*)workspace(ctx, S_Q, vb);
  cplx<T>* z = o.precond == IOBM_PC_NONE ? r : (cplx<T>*)workspace(ctx, S_Z, vb);
  cplx<T>* pf = o.precond == IOBM_PC_LATERAL_FFT ? (cplx<T>*)workspace(ctx, S_PF, vb) : nullptr;
  // point blocks per group of a Gram launch: about 512 blocks in all
  auto gram_blocks = [](int ngroups) { return std::min(128, std::max(16, 512 / std::max(1, ngroups))); };
  // group ids: the energies' groups, then the halves of split groups (one
  // new id per split, at most nb groups at any time)
  const int gcap = std::max(ng, nb);
  // packed Gram partials: nblk * 4 * sum s^2 doubles.  With G groups in a
  // launch, sum s^2 <= min(64^2 G, 64 nb): for G <= 32, nblk <= 512 / G or
  // 128, so nblk sum s^2 <= min(512 * 64^2, 128 * 64 nb); beyond, nblk = 16
  // and nblk sum s^2 <= 16 * 64 nb
  const size_t gpart_n = std::max(std::min<size_t>((size_t)512 * 64 * 64, (size_t)128 * 64 * nb), (size_t)16 * 64 * nb);
  double* gpart = (double*)workspace(ctx, S_BLK_PART, gpart_n * 4 * sizeof(double));
  const size_t gmat = (size_t)64 * 64;
  zd* gm = (zd*)workspace(ctx, S_BLK_G, 6 * (size_t)gcap * gmat * sizeof(zd));
  zd* G1 = gm;
  zd* G2 = gm + (size_t)gcap * gmat;
  zd* G2n = gm + 2 * (size_t)gcap * gmat;
  zd* AL = gm + 3 * (size_t)gcap * gmat;
  zd* BE = gm + 4 * (size_t)gcap * gmat;
  zd* GW = gm + 5 * (size_t)gcap * gmat;
  const int nchunk = (int)std::min<long long>(256, (vol + 63) / 64);
  Partial* n2p = (Partial*)workspace(ctx, S_BLK_N2, (size_t)nb * nchunk * sizeof(Partial));
  const int nblk = dot_blocks(ctx);
  Partial* part = (Partial*)workspace(ctx, S_PART, (size_t)nb * nblk * sizeof(Partial));
  Partial* part_rn = (Partial*)workspace(ctx, S_PARTR, (size_t)nb * PQ_SLOTS * sizeof(Partial));
  const size_t nb8 = ((size_t)nb + 1) & ~(size_t)1, ng8 = ((size_t)gcap + 1) & ~(size_t)1;
  char* sc = (char*)workspace(ctx, S_SCAL, (size_t)nb * 3 * sizeof(zd) + nb8 * (2 * sizeof(double) + 3 * sizeof(int)) +
                                             2 * ng8 * sizeof(int) + 64);
  zd* rho = (zd*)sc;
  zd* alpha = rho + nb;  // zero: x += d + 0 p at a refresh
  zd* beta = alpha + nb;
  double* rn2 = (double*)(beta + nb);
  int* flag = (int*)(rn2 + nb);
  double* tn2 = (double*)(flag + nb8);
  int* xset = (int*)(tn2 + nb8);
  int* dlive = xset + nb8;
  int* gflag = dlive + nb8;  // [2][gcap]: breakdown of the alpha and the beta solve
  const size_t chk = (size_t)nb * sizeof(double);
  char* rbh = (char*)pinned_readback(ctx, chk + nb8 * sizeof(int) + (size_t)nb * sizeof(double) + 2 * ng8 * sizeof(int) + 64);
  const double* rn2_h = (const double*)rbh;
  int* gflag_h = (int*)(rbh + chk);
  double* tn2_pin = (double*)(rbh + chk + 2 * ng8 * sizeof(int));
  if (ctx->kb.ncen > 0) (void)kb_scratch(ctx, kb_proj_bytes(ctx, nb));
  const ModeData* modes = ctx->modes_d;
  const bool lowp = sizeof(T) == sizeof(float);
  const double tol2 = o.tol * o.tol;
  const double delta2 = lowp ? o.inner_tol * o.inner_tol : 0.0;
  const int check = o.check_every > 0 ? o.check_every : 2;  // 0 (scheduled checks): every 2 iterations here

  auto precond = [&](int n, const int* ld) {
    if (o.precond == IOBM_PC_TRUNCATED_LAPLACIAN) HIPCHK(launch_precond_laplacian<T>(ctx, o.alpha, r, z, n, ld));
    else if (o.precond == IOBM_PC_LATERAL_FFT) HIPCHK(launch_precond_fft<T>(ctx, r, z, pf, n, e_d, modes, ld));
    else if (o.precond == IOBM_PC_JACOBI) HIPCHK(launch_precond_jacobi<T>(ctx, r, z, n, e_d, E_d, ld));
  };
  auto read_tn2 = [&](std::vector<double>& dst) {
    HIPCHK(hipMemcpyAsync(tn2_pin, tn2, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    memcpy(dst.data(), tn2_pin, nb * sizeof(double));
  };
  // group lists on the device: [gid | goff | gsize | poff | cols] in one upload
  struct Groups {
    int n = 0, ncols = 0;
    const int *gid = nullptr, *goff = nullptr, *gsize = nullptr, *poff = nullptr, *cols = nullptr;
  };
  auto make_groups = [&](const std::vector<int>& gl, const std::vector<std::vector<int>>& gc, int region) {
    Groups G;
    G.n = (int)gl.size();
    std::vector<int> buf(4 * G.n);
    int sq = 0;
    for (int k = 0; k < G.n; ++k) {
      const int sz = (int)gc[gl[k]].size();
      buf[k] = gl[k];
      buf[G.n + k] = G.ncols;
      buf[2 * G.n + k] = sz;
      buf[3 * G.n + k] = sq;
      G.ncols += sz;
      sq += sz * sz;
    }
    for (int k = 0; k < G.n; ++k) buf.insert(buf.end(), gc[gl[k]].begin(), gc[gl[k]].end());
    const int* dptr = upload(ctx, S_IDX, buf, (size_t)region * 8192);
    G.gid = dptr;
    G.goff = dptr + G.n;
    G.gsize = dptr + 2 * G.n;
    G.poff = dptr + 3 * G.n;
    G.cols = dptr + 4 * G.n;
    return G;
  };
  // (re)start the block recursion of the listed groups: Z = M R, G2 = R^T Z, P = Z
  auto start_groups = [&](const Groups& S) {
    if (S.n == 0) return;
    precond(S.ncols, S.cols);
    HIPCHK(launch_gram<T>(ctx, r, z, S.n, S.cols, S.goff, S.gsize, S.gid, S.poff, gpart, gram_blocks(S.n), G2,
                          S.ncols));
    HIPCHK((launch_convert<T, T>(ctx, z, pa, S.ncols, S.cols)));
  };

  // start: x = 0, d = 0, r = b; the refresh's partial slots start at zero
  // (slots past the stencil chunks and the electrode faces are never written)
  HIPCHK(hipMemsetAsync(part_rn, 0, (size_t)nb * PQ_SLOTS * sizeof(Partial), ctx->stream));
  HIPCHK((launch_convert<double, double>(ctx, nullptr, x, nb, all_d)));
  HIPCHK((launch_convert<T, T>(ctx, nullptr, d, nb, all_d)));
  HIPCHK(hipMemsetAsync(alpha, 0, nb * sizeof(zd), ctx->stream));
  HIPCHK(hipMemsetD32Async((hipDeviceptr_t)xset, 1, 2 * nb8, ctx->stream));  // xset and dlive: x and d hold data
  HIPCHK(launch_face_norm2(ctx, b, nb, all_d, part));
  HIPCHK(launch_finish2(ctx, rho, alpha, beta, tn2, flag, part, 1, nullptr, 0, FIN_NORM, nb, all_d));
  std::vector<double> bn2(nb), tn2_h(nb);
  read_tn2(bn2);
  tn2_h = bn2;
  HIPCHK(launch_init_r<T>(ctx, b, r, nb, all_d));
  std::vector<std::vector<int>> gc(gcap);
  std::vector<int> glist;
  int next_gid = ng;
  for (int g = 0; g < ng; ++g) {
    for (int i = gfirst[g]; i < gfirst[g] + gsz[g]; ++i)
      if (bn2[i] > 0) gc[g].push_back(i);
    if (!gc[g].empty()) glist.push_back(g);
  }
  std::vector<double> maxr2(bn2), best(bn2);
  std::vector<int> stall(nb, 0);
  std::vector<char> want(nb, 0);  // the column itself asked for the group's refresh
  Groups A = make_groups(glist, gc, 8);
  start_groups(A);
  int it = 0;
  while (A.n > 0) {
    for (int k = 0; k < check; ++k) {
      HIPCHK(launch_apply<T>(ctx, pa, q, A.ncols, E_d, e_d, modes, A.cols));
      HIPCHK(launch_gram<T>(ctx, pa, q, A.n, A.cols, A.goff, A.gsize, A.gid, A.poff, gpart, gram_blocks(A.n), G1,
                            A.ncols));
      HIPCHK(launch_small_solve(ctx, A.n, A.gsize, A.gid, G1, G2, GW, AL, gflag));
      HIPCHK((launch_block_update<T, T>(ctx, d, pa, nullptr, AL, A.n, A.cols, A.goff, A.gsize, A.gid, nchunk, 0,
                                        nullptr, A.ncols)));
      HIPCHK((launch_block_update<T, T>(ctx, r, q, nullptr, AL, A.n, A.cols, A.goff, A.gsize, A.gid, nchunk, 1, n2p,
                                        A.ncols)));
      precond(A.ncols, A.cols);
      HIPCHK(launch_gram<T>(ctx, r, z, A.n, A.cols, A.goff, A.gsize, A.gid, A.poff, gpart, gram_blocks(A.n), G2n,
                            A.ncols));
      HIPCHK(launch_small_solve(ctx, A.n, A.gsize, A.gid, G2, G2n, GW, BE, gflag + ng8));
      std::swap(G2, G2n);
      HIPCHK((launch_block_update<T, T>(ctx, pb, pa, z, BE, A.n, A.cols, A.goff, A.gsize, A.gid, nchunk, 2, nullptr,
                                        A.ncols)));
      std::swap(pa, pb);
    }
    it += check;
    HIPCHK(launch_finish2(ctx, rho, alpha, beta, rn2, flag, n2p, nchunk, nullptr, 0, FIN_NORM, A.ncols, A.cols));
    HIPCHK(hipMemcpyAsync(rbh, rn2, chk, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(gflag_h, gflag, 2 * ng8 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    // groups to refresh: a group goes when any of its columns asks for it
    // (its own target, replacement factor, divergence) or a Gram solve broke
    // down; maxr2 tracks each column's largest iterated residual since its
    // last refresh
    std::vector<int> upd_g, upd_c;
    for (int g : glist) {
      const bool brk = gflag_h[g] || gflag_h[ng8 + g];
      bool go = brk, all_conv = true;
      for (int i : gc[g]) {
        out.iters[i] += check;
        const double r2 = rn2_h[i];
        const bool conv = r2 <= 0.25 * tol2 * bn2[i];
        const bool w = !(r2 == r2) || r2 > 1e4 * maxr2[i] || r2 <= delta2 * maxr2[i] || out.iters[i] >= o.max_iter;
        all_conv = all_conv && conv;
        want[i] = w || brk || conv;
        if (!w) maxr2[i] = std::max(maxr2[i], r2);
        go = go || w;
      }
      go = go || all_conv;
      if (go) {
        upd_g.push_back(g);
        upd_c.insert(upd_c.end(), gc[g].begin(), gc[g].end());
      }
    }
    if (upd_g.empty()) continue;
    // refresh: x += d, d = 0, r = b - A x in FP64 (stored in the iteration precision)
    {
      int* ld = upload(ctx, S_IDX, upd_c, 7 * 8192);
      const int n = (int)upd_c.size();
      HIPCHK(launch_accumulate<T>(ctx, x, d, pa, alpha, xset, dlive, n, ld, 0, 0));
      HIPCHK((launch_convert<T, T>(ctx, nullptr, d, n, ld)));
      if (ctx->kb.ncen == 0) {
        HIPCHK(launch_refresh<T>(ctx, x, b, rhi, r, n, E_d, e_d, modes, ld, part_rn));
        HIPCHK(launch_finish2(ctx, rho, alpha, beta, tn2, flag, part_rn, PQ_SLOTS, nullptr, 0, FIN_NORM, n, ld));
      } else {
        HIPCHK(launch_apply<double>(ctx, x, rhi, n, E_d, e_d, modes, ld));
        HIPCHK(launch_residual<double>(ctx, b, rhi, n, ld));
        HIPCHK(launch_dot<double>(ctx, rhi, rhi, n, ld, part));
        HIPCHK(launch_finish2(ctx, rho, alpha, beta, tn2, flag, part, nblk, nullptr, 0, FIN_NORM, n, ld));
        HIPCHK((launch_convert<T, double>(ctx, rhi, r, n, ld)));
      }
      read_tn2(tn2_h);
    }
    std::vector<int> restart_g;
    for (int g : upd_g) {
      const bool brk = gflag_h[g] || gflag_h[ng8 + g];
      const bool split = brk && gc[g].size() > 1;
      std::vector<int> keep;
      for (int i : gc[g]) {
        out.refin[i] += 1;
        const double t2 = tn2_h[i];
        if (t2 <= tol2 * bn2[i]) continue;
        if (out.iters[i] >= o.max_iter) { out.status[i] = IOBM_E_NOT_CONVERGED; continue; }
        // a refresh the column asked for must improve its true residual
        // (six in a row without a fourfold gain end it); one triggered by
        // another column of the group does not count against it, and a
        // split gives the columns a fresh start
        if (t2 < 0.25 * best[i] || split) { best[i] = std::min(best[i], t2); stall[i] = 0; }
        else if (want[i] && ++stall[i] >= 6) {
          out.status[i] = brk ? IOBM_E_BREAKDOWN : IOBM_E_NOT_CONVERGED;
          continue;
        }
        maxr2[i] = t2;
        keep.push_back(i);
      }
      if (split && keep.size() > 1) {
        // every column but the first moves to a group of its own (new ids
        // never run out: each split adds at most its columns - 1 groups)
        std::vector<int> stay(1, keep[0]);
        for (size_t k = 1; k < keep.size(); ++k) {
          if (next_gid >= gcap) { stay.push_back(keep[k]); continue; }
          const int ng2 = next_gid++;
          gc[ng2].assign(1, keep[k]);
          restart_g.push_back(ng2);
        }
        keep = stay;
      }
      gc[g] = keep;
      if (!keep.empty()) restart_g.push_back(g);
    }
    // groups in the order of their first column (deterministic launch order)
    std::vector<int> nl;
    for (int g = 0; g < next_gid; ++g)
      if (!gc[g].empty()) nl.push_back(g);
    std::sort(nl.begin(), nl.end(), [&](int a, int b) { return gc[a][0] < gc[b][0]; });
    std::sort(restart_g.begin(), restart_g.end(), [&](int a, int b) { return gc[a][0] < gc[b][0]; });
    glist = nl;
    A = make_groups(glist, gc, 8);
    start_groups(make_groups(restart_g, gc, 16));
  }
  (void)it;
  for (int i = 0; i < nb; ++i) {
    out.rel[i] = bn2[i] > 0 ? sqrt(tn2_h[i] / bn2[i]) : 0.0;
    if (out.status[i] == IOBM_OK && bn2[i] > 0 && tn2_h[i] > tol2 * bn2[i]) out.status[i] = IOBM_E_NOT_CONVERGED;
  }
}

void solve_batch(iobm_ctx ctx, const iobm_solve_opts& o, const Batch& B, const zd* b, zd* x, SolveOut& out) {
  if (o.block) {
    // the complex64 block recurrence loses the small differences between
    // the nearly dependent residual columns of a group and diverges after a
    // few replacements: block COCG runs in complex128
    if (o.precision != IOBM_C128) {
      ctx->err = "block COCG runs in complex128 only (opts.precision = IOBM_C128)";
      throw Fail{IOBM_E_UNSUPPORTED};
    }
    solve_block_batch<double>(ctx, o, B, b, x, out);
    return;
  }
  if (o.precision == IOBM_C64_REFINED) solve_rhs_batch<float>(ctx, o, B, b, x, out);
  else solve_rhs_batch<double>(ctx, o, B, b, x, out);
}

void validate_opts(iobm_ctx ctx, const iobm_solve_opts* o) {
  if (!o) { ctx->err = "opts is NULL"; throw Fail{IOBM_E_INVALID_ARG}; }
  if (o->precision != IOBM_C128 && o->precision != IOBM_C64_REFINED) {
    ctx->err = "unknown precision"; throw Fail{IOBM_E_INVALID_ARG};
  }
  if (o->precond < IOBM_PC_NONE || o->precond > IOBM_PC_JACOBI) {
    ctx->err = "unknown preconditioner"; throw Fail{IOBM_E_INVALID_ARG};
  }
  if (!(o->tol > 0 && o->tol < 1) || !(o->inner_tol > 0 && o->inner_tol < 1) || o->max_iter < 1 ||
      o->check_every < 0 || (o->keep_direction != 0 && o->keep_direction != 1) || (o->graph != 0 && o->graph != 1) || (o->block != 0 && o->block != 1) ||
      (o->side != 0 && o->side != 1) || !(o->alpha > 0) || !isfinite(o->alpha)) {
    ctx->err = "invalid solver option (tol, inner_tol in (0,1), max_iter >= 1, check_every >= 0, side 0/1, "
               "keep_direction 0/1, graph 0/1, block 0/1, alpha > 0)";
    throw Fail{IOBM_E_INVALID_ARG};
  }
}

// Build the request list and the real-lateral-basis batch.
void plan_requests(iobm_ctx ctx, int nE, const double* E, const int* ninc, const int* inc, Batch& B,
                   Request& Q) {
  const GridDev& g = ctx->g;
  int pos = 0;
  for (int e = 0; e < nE; ++e) {
    std::vector<int> ids;
    const int* fl = &ctx->mode_flags_h[(size_t)e * g.nxy];
    if (ninc[e] < 0) {
      for (int m = 0; m < g.nxy; ++m)
        if (fl[m] & MODE_OPEN) ids.push_back(m);
    } else {
      for (int k = 0; k < ninc[e]; ++k) {
        int m = inc[pos++];
        if (m < 0 || m >= g.nxy || !(fl[m] & MODE_OPEN)) {
          char buf[128];
          snprintf(buf, sizeof buf, "channel %d is not open at energy %.12g", m, E[e]);
          ctx->err = buf;
          throw Fail{IOBM_E_INVALID_ARG};
        }
        ids.push_back(m);
      }
    }
    std::map<std::pair<int, int>, int> basis;  // (canonical mode, kind) -> rhs
    auto get = [&](int m, int kind) {
      auto key = std::make_pair(m, kind);
      auto it = basis.find(key);
      if (it != basis.end()) return it->second;
      int id = B.n++;
      B.e.push_back(e);
      B.E.push_back(E[e]);
      B.mode.push_back(m);
      B.kind.push_back(kind);
      basis[key] = id;
      return id;
    };
    for (int m : ids) {
      int nm = neg_mode(g, m);
      int canon = std::min(m, nm);
      Q.e.push_back(e);
      Q.mode.push_back(m);
      if (nm == m) {
        Q.c.push_back(get(m, 1));
        Q.s.push_back(-1);
        Q.sgn.push_back(0);
      } else {
        Q.c.push_back(get(canon, 1));
        Q.s.push_back(get(canon, 2));
        Q.sgn.push_back(m == canon ? 1 : -1);
      }
    }
  }
}

// One batched solve of every requested (energy, channel) pair and its
// readout.  The device results (solutions x, per-request amplitudes t_out
// and r_out [nreq][nxy], T and R in TR [2 nreq]) live in the workspace pool
// until the next call; the request lists are on the device (qc, qs, qg).
struct SolveRun {
  Batch B;
  Request Q;
  SolveOut so;
  zd* x = nullptr;
  zd* t_out = nullptr;
  zd* r_out = nullptr;
  double* TR = nullptr;
  int *qc = nullptr, *qs = nullptr, *qg = nullptr;
};

void run_solve(iobm_ctx ctx, const iobm_solve_opts& o, int nE, const double* E, const int* ninc, const int* inc,
               SolveRun& run) {
  plan_requests(ctx, nE, E, ninc, inc, run.B, run.Q);
  const int nb = run.B.n, nreq = (int)run.Q.e.size();
  const long long vol = ctx->g.npts;
  const int nxy = ctx->g.nxy;
  zd* b = (zd*)workspace(ctx, S_B, (size_t)nb * vol * sizeof(zd));
  run.x = (zd*)workspace(ctx, S_XHI, (size_t)nb * vol * sizeof(zd));
  {
    int* e_d = upload(ctx, S_IDX, run.B.e, 0);
    int* m_d = upload(ctx, S_IDX, run.B.mode, 16 * 1024);
    int* k_d = upload(ctx, S_IDX, run.B.kind, 32 * 1024);
    HIPCHK(launch_rhs(ctx, nb, e_d, m_d, k_d, o.side, ctx->modes_d, b, true));
  }
  solve_batch(ctx, o, run.B, b, run.x, run.so);
  // readout of every basis solution, then combination into channels
  zd* amp = (zd*)workspace(ctx, S_AMP, (size_t)(2 * nb + 2 * nreq) * nxy * sizeof(zd));
  zd* amp_near = amp;
  zd* amp_far = amp + (size_t)nb * nxy;
  run.t_out = amp + (size_t)2 * nb * nxy;
  run.r_out = run.t_out + (size_t)nreq * nxy;
  run.TR = (double*)workspace(ctx, S_TR, (size_t)2 * nreq * sizeof(double) + 64);
  int* e_d = upload(ctx, S_IDX, run.B.e, 0);
  HIPCHK(launch_readout(ctx, nb, o.side, run.x, ctx->modes_d, e_d, amp_near, amp_far));
  int* qe = upload(ctx, S_IDX, run.Q.e, 16 * 1024);
  int* qm = upload(ctx, S_IDX, run.Q.mode, 24 * 1024);
  run.qc = upload(ctx, S_IDX, run.Q.c, 32 * 1024);
  run.qs = upload(ctx, S_IDX, run.Q.s, 40 * 1024);
  run.qg = upload(ctx, S_IDX, run.Q.sgn, 48 * 1024);
  HIPCHK(launch_combine(ctx, nreq, qe, qm, run.qc, run.qs, run.qg, ctx->modes_d, amp_near, amp_far, run.t_out,
                        run.r_out, run.TR, run.TR + nreq));
}

// Per-request statistics (cos + sin solves of a +-G pair summed) and the
// worst status.
iobm_status request_stats(const SolveRun& run, const std::vector<double>& TRh, iobm_solve_stat* st) {
  const int nreq = (int)run.Q.e.size();
  iobm_status worst = IOBM_OK;
  const SolveOut& so = run.so;
  for (int c = 0; c < nreq; ++c) {
    int ic = run.Q.c[c], is = run.Q.s[c];
    int status = so.status[ic];
    if (is >= 0 && so.status[is] != IOBM_OK) status = so.status[is];
    if (status != IOBM_OK) worst = (iobm_status)status;
    if (st) {
      st[c].iters = so.iters[ic] + (is >= 0 ? so.iters[is] : 0);
      st[c].refinements = so.refin[ic] + (is >= 0 ? so.refin[is] : 0);
      st[c].status = status;
      st[c].pad_ = 0;
      st[c].rel_residual = std::max(so.rel[ic], is >= 0 ? so.rel[is] : 0.0);
      st[c].flux_error = TRh[c] + TRh[nreq + c] - 1.0;
    }
  }
  return worst;
}

// ------------------------------------------- lateral Bloch vector kappa
// States of a solve at kappa != 0, in pairs: slot 2k at +kappa (mode-table
// entry e, incident channel mu), slot 2k+1 its partner at -kappa (entry
// nE + e, channel -mu), both incident from the same side.
struct PairBatch {
  int n = 0;               // slots (two per pair)
  std::vector<int> e;      // mode-table entry per slot
  std::vector<double> E;   // energy per slot
  std::vector<int> mode;   // incident channel per slot
  std::vector<int> sgn;    // +1 at +kappa, -1 at -kappa
};

enum { BL_ALPHA = 0, BL_BETA = 1, BL_RESTART = 2 };

// Preconditioned biconjugate gradients with the bilinear form on pairs
// (the primary solves A(kappa) x = b, the shadow A(kappa)^T y = c with
// A(kappa)^T = A(-kappa) and the preconditioner P(kappa)^T = P(-kappa)):
//   q = A p, q~ = A^T p~;  alpha = rho / (p~^T q);
//   d += alpha p, d~ += alpha p~;  r -= alpha q, r~ -= alpha q~;
//   z = P r, z~ = P^T r~;  rho' = r~^T z;  beta = rho' / rho;
//   p = z + beta p, p~ = z~ + beta p~,
// in the iteration precision T on the correction d of the FP64 solution x
// (complex128: d is x itself), every inner product summed in FP64 in a
// fixed order.  One operator pass forms the direction (p = z + beta p into
// the other of two buffers), applies A to it and adds the previous step's
// alpha p to d, so a step's d update stays pending until the next pass, or
// until a restart or a stop folds it in (x += d + alpha p).  A pair is
// restarted from its true residual (that fold, d = 0, r = b - A x with the
// complex128 operator, then p = z) when its recursive residuals both reach
// tol ||b||, or (complex64) have both fallen by opts.inner_tol since its
// last restart, or when it broke down (vanishing rho or p~^T q) or
// diverged.  It is done when both true residuals are below tol ||b||.  The
// operators run in the gauge u = exp(-i kappa.r) psi.
template <typename T>
void solve_pair_batch(iobm_ctx ctx, const iobm_solve_opts& o, const BlochPhase& ph, const PairBatch& B, const zd* b,
                      zd* x, SolveOut& out) {
  constexpr bool lowp = sizeof(T) == sizeof(float);
  const int ns = B.n, np = ns / 2;
  const long long vol = ctx->g.npts;
  out.iters.assign(ns, 0);
  out.refin.assign(ns, 0);
  out.status.assign(ns, IOBM_OK);
  out.rel.assign(ns, 0.0);
  if (np == 0) return;
  const size_t vb = (size_t)ns * vol * sizeof(cplx<T>);
  int* e_d = upload(ctx, S_IDX, B.e, 0);
  double* E_d = upload(ctx, S_IDX, B.E, 16 * 1024);
  int* sg_d = upload(ctx, S_IDX, B.sgn, 32 * 1024);
  cplx<T>* r = (cplx<T>*)workspace(ctx, S_R, vb);
  cplx<T>* pc = (cplx<T>*)workspace(ctx, S_P, vb);   // the last step's direction (its alpha p pending)
  cplx<T>* po = (cplx<T>*)workspace(ctx, S_P2, vb);  // the next step's
  cplx<T>* q = (cplx<T>*)workspace(ctx, S_Q, vb);
  cplx<T>* z = o.precond == IOBM_PC_NONE ? r : (cplx<T>*)workspace(ctx, S_Z, vb);
  cplx<T>* pf = o.precond == IOBM_PC_LATERAL_FFT ? (cplx<T>*)workspace(ctx, S_PF, vb) : nullptr;
  // the correction (complex128: x itself), and the FP64 face planes of a
  // restart's residual (complex128: in q, which the next pass overwrites)
  cplx<T>* d = lowp ? (cplx<T>*)workspace(ctx, S_D, vb) : (cplx<T>*)x;
  zd* rface = lowp ? (zd*)workspace(ctx, S_RHI, (size_t)ns * vol * sizeof(zd)) : (zd*)q;
  const int nblk = dot_blocks(ctx);
  Partial* pd = (Partial*)workspace(ctx, S_PART, (size_t)np * nblk * sizeof(Partial));
  Partial* pn = (Partial*)workspace(ctx, S_PARTR, (size_t)ns * nblk * sizeof(Partial));
  Partial* pq = (Partial*)workspace(ctx, S_PARTN, (size_t)ns * PQ_SLOTS * sizeof(Partial));
  char* sc = (char*)workspace(ctx, S_SCAL, (size_t)np * 3 * sizeof(zd) + (size_t)ns * sizeof(double) +
                                                  (size_t)np * sizeof(int) + 64);
  zd* rho = (zd*)sc;
  zd* alpha = rho + np;
  zd* beta = alpha + np;
  double* rn2 = (double*)(beta + np);
  int* flag = (int*)(rn2 + ns);
  const size_t rb_bytes = (size_t)ns * sizeof(double) + (size_t)np * sizeof(int);
  char* rbh = (char*)pinned_readback(ctx, rb_bytes + 64);
  const double* rn2_h = (const double*)rbh;
  const int* flag_h = (const int*)(rbh + (size_t)ns * sizeof(double));
  const double tol2 = o.tol * o.tol;
  const double delta2 = lowp ? o.inner_tol * o.inner_tol : 0.0;
  const int check = o.check_every > 0 ? o.check_every : 1;  // 0 (scheduled checks): every iteration here
  HIPCHK(hipMemsetAsync(x, 0, (size_t)ns * vol * sizeof(zd), ctx->stream));
  if (lowp) HIPCHK(hipMemsetAsync(d, 0, vb, ctx->stream));
  // rho, alpha, beta: nothing pending before the first restart
  HIPCHK(hipMemsetAsync(rho, 0, (size_t)np * 3 * sizeof(zd), ctx->stream));
  cplx<T>* dfold = lowp ? d : nullptr;  // complex128: the recurrence updates x itself
  int nfresh = 0;                       // slots restarted since their last step

  // device lists of the pairs in `pairs_h` (pair ids): their slots (2k,
  // 2k+1 in pair order) and their primary slots
  int *sl_d = nullptr, *pl_d = nullptr;
  auto set_lists = [&](const std::vector<int>& pairs_h) {
    std::vector<int> sl, pl;
    for (int k : pairs_h) {
      sl.push_back(2 * k);
      sl.push_back(2 * k + 1);
      pl.push_back(2 * k);
    }
    sl_d = upload(ctx, S_IDX, sl, 40 * 1024);
    pl_d = upload(ctx, S_IDX, pl, 48 * 1024);
  };
  auto precond = [&](int nsl) {
    if (o.precond == IOBM_PC_TRUNCATED_LAPLACIAN)
      HIPCHK(launch_bloch_laplacian<T>(ctx, ph, o.alpha, r, z, nsl, sg_d, sl_d));
    else if (o.precond == IOBM_PC_LATERAL_FFT)
      HIPCHK(launch_precond_fft<T>(ctx, r, z, pf, nsl, e_d, ctx->modes_d, sl_d, nullptr));
    else if (o.precond == IOBM_PC_JACOBI)
      HIPCHK(launch_precond_jacobi<T>(ctx, r, z, nsl, e_d, E_d, sl_d, nullptr));
  };
  // x += d + alpha p, r = b - A x (one complex128 operator pass that writes
  // r in the iteration precision), z = P r, rho = r~^T z, alpha = beta = 0
  // (the next pass takes p = z) for the listed pairs
  auto restart = [&](int npr) {
    HIPCHK(launch_bloch_settle<T>(ctx, x, dfold, pc, alpha, 2 * npr, sl_d, nblk));
    HIPCHK(launch_bloch_refresh<T>(ctx, ph, x, b, rface, r, 2 * npr, E_d, e_d, sg_d, sl_d, pq));
    precond(2 * npr);
    HIPCHK(launch_bloch_dot<T>(ctx, r, z, npr, pl_d, pd, nblk));
    HIPCHK(launch_bloch_scalars(ctx, BL_RESTART, npr, pl_d, pd, pq, nblk, rho, alpha, beta, rn2, flag));
  };
  auto iterate = [&](int npr) {
    const BlochFuse<T> F{z, pc, po, d, beta, alpha, nfresh};
    HIPCHK(launch_bloch_apply_fused<T>(ctx, ph, F, q, 2 * npr, E_d, e_d, sg_d, sl_d));
    std::swap(pc, po);
    nfresh = 0;
    HIPCHK(launch_bloch_dot<T>(ctx, pc, q, npr, pl_d, pd, nblk));
    HIPCHK(launch_bloch_scalars(ctx, BL_ALPHA, npr, pl_d, pd, pn, nblk, rho, alpha, beta, rn2, flag));
    HIPCHK(launch_bloch_update<T>(ctx, r, q, alpha, 2 * npr, sl_d, pn, nblk));
    precond(2 * npr);
    HIPCHK(launch_bloch_dot<T>(ctx, r, z, npr, pl_d, pd, nblk));
    HIPCHK(launch_bloch_scalars(ctx, BL_BETA, npr, pl_d, pd, pn, nblk, rho, alpha, beta, rn2, flag));
  };
  auto read_back = [&]() {
    HIPCHK(hipMemcpyAsync(rbh, rn2, (size_t)ns * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(rbh + (size_t)ns * sizeof(double), flag, (size_t)np * sizeof(int), hipMemcpyDeviceToHost,
                          ctx->stream));
    stream_sync(ctx);
  };

  std::vector<int> act(np);
  for (int k = 0; k < np; ++k) act[k] = k;
  set_lists(act);
  restart(np);  // x = 0: r = b
  nfresh = ns;
  read_back();
  std::vector<double> bn2(rn2_h, rn2_h + ns), last(bn2);
  std::vector<int> it(np, 0), rs(np, 0);
  auto finish = [&](int k, int status) {
    for (int s2 = 0; s2 < 2; ++s2) {
      const int sl = 2 * k + s2;
      out.iters[sl] = it[k];
      out.refin[sl] = rs[k];
      out.status[sl] = status;
      out.rel[sl] = bn2[sl] > 0 ? sqrt(rn2_h[sl] / bn2[sl]) : 0.0;
    }
  };
  auto pair_conv = [&](int k) {
    return rn2_h[2 * k] <= tol2 * bn2[2 * k] && rn2_h[2 * k + 1] <= tol2 * bn2[2 * k + 1];
  };
  // both slots at the target or fallen by the replacement factor since the
  // last restart (complex64)
  auto pair_replace = [&](int k) {
    for (int s2 = 0; s2 < 2; ++s2) {
      const int sl = 2 * k + s2;
      if (!(rn2_h[sl] <= std::max(tol2 * bn2[sl], delta2 * last[sl]))) return false;
    }
    return true;
  };
  {  // right-hand sides that vanish, or a first rho that vanishes
    std::vector<int> keep;
    for (int k : act) {
      if (pair_conv(k)) finish(k, IOBM_OK);
      else if (flag_h[k]) finish(k, IOBM_E_BREAKDOWN);
      else keep.push_back(k);
    }
    if (keep.size() != act.size()) {
      act = keep;
      if (!act.empty()) set_lists(act);
    }
  }
  const int max_restarts = 1000;
  while (!act.empty()) {
    const int npr = (int)act.size();
    for (int c2 = 0; c2 < check; ++c2) iterate(npr);
    for (int k : act) it[k] += check;
    read_back();
    std::vector<int> keep, redo, stop;
    for (int k : act) {
      const double a = rn2_h[2 * k], c3 = rn2_h[2 * k + 1];
      const bool bad = flag_h[k] || !std::isfinite(a) || !std::isfinite(c3) || a > 1e20 * bn2[2 * k] ||
                       c3 > 1e20 * bn2[2 * k + 1];
      if (bad || pair_conv(k) || pair_replace(k)) redo.push_back(k);
      else if (it[k] >= o.max_iter) {
        finish(k, IOBM_E_NOT_CONVERGED);
        stop.push_back(k);
      } else keep.push_back(k);
    }
    if (!stop.empty()) {  // fold in the pending correction of the pairs that stop here
      set_lists(stop);
      HIPCHK(launch_bloch_settle<T>(ctx, x, dfold, pc, alpha, 2 * (int)stop.size(), sl_d, nblk));
    }
    if (!redo.empty()) {
      set_lists(redo);
      restart((int)redo.size());
      read_back();
      for (int k : redo) {
        ++rs[k];
        last[2 * k] = rn2_h[2 * k];
        last[2 * k + 1] = rn2_h[2 * k + 1];
        if (pair_conv(k)) finish(k, IOBM_OK);
        else if (flag_h[k] || rs[k] >= max_restarts) finish(k, IOBM_E_BREAKDOWN);
        else if (it[k] >= o.max_iter) finish(k, IOBM_E_NOT_CONVERGED);
        else {
          keep.push_back(k);
          nfresh += 2;
        }
      }
    }
    std::sort(keep.begin(), keep.end());
    if (keep != act || !redo.empty()) {
      act = keep;
      if (!act.empty()) set_lists(act);
    }
  }
  // every pair ended right after a restart or a stop, each of which folded
  // in its pending correction: x holds the solution
}

}  // namespace

int prof_start(iobm_ctx c, int cls) {
  if (!(c->prof_mask & (1 << cls))) return -1;
  if (2 * c->prof_used + 2 > c->prof_ev.size()) {
    for (int k = 0; k < 128; ++k) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) return -1;
      c->prof_ev.push_back(ev);
    }
  }
  const size_t rec = c->prof_used++;
  if (c->prof_cls.size() <= rec) {
    c->prof_cls.resize(rec + 1);
    c->prof_bytes.resize(rec + 1);
  }
  c->prof_cls[rec] = cls;
  c->prof_bytes[rec] = 0;
  (void)hipEventRecord(c->prof_ev[2 * rec], c->stream);
  return (int)rec;
}

void prof_stop(iobm_ctx c, int rec, double alg_bytes) {
  if (rec < 0 || (size_t)rec >= c->prof_used) return;
  (void)hipEventRecord(c->prof_ev[2 * rec + 1], c->stream);
  c->prof_bytes[rec] = alg_bytes;
}

double* kb_scratch(iobm_ctx c, size_t bytes) {
  try {
    return (double*)workspace(c, S_KB, bytes);
  } catch (Fail&) {
    return nullptr;
  }
}

// ======================================================================= ABI
extern "C" {

void iobm_default_opts(iobm_solve_opts* o) {
  if (!o) return;
  o->precision = IOBM_C64_REFINED;
  o->precond = IOBM_PC_LATERAL_FFT;
  o->alpha = 1.8;
  o->tol = 1e-10;
  o->inner_tol = 1e-3;
  o->max_iter = 50000;
  o->side = 0;
  o->check_every = 0;
  o->keep_direction = 0;
  o->graph = 0;
  o->block = 0;
  o->pad_ = 0;
}

const char* iobm_status_str(iobm_status s) {
  switch (s) {
    case IOBM_OK: return "ok";
    case IOBM_E_INVALID_ARG: return "invalid argument";
    case IOBM_E_BAD_STATE: return "bad state";
    case IOBM_E_OOM: return "out of device memory";
    case IOBM_E_DEVICE: return "device error";
    case IOBM_E_NOT_CONVERGED: return "not converged";
    case IOBM_E_BREAKDOWN: return "Krylov breakdown";
    case IOBM_E_AT_THRESHOLD: return "energy at a channel threshold";
    case IOBM_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* iobm_last_error(iobm_ctx ctx) { return ctx ? ctx->err.c_str() : "no context"; }

iobm_status iobm_create(const iobm_grid* g, void* stream, iobm_ctx* out) {
  if (!g || !out) return IOBM_E_INVALID_ARG;
  *out = nullptr;
  // a lateral period of at least nf points: a neighbour at distance n <= nf
  // wraps across the cell at most once
  if (g->nf < 1 || g->nf > 3 || g->nx < std::max(2, g->nf) || g->ny < std::max(2, g->nf) || g->nz < 2 * g->nf ||
      !(g->hx > 0) ||
      !(g->hy > 0) || !(g->hz > 0) || !isfinite(g->hx) || !isfinite(g->hy) || !isfinite(g->hz))
    return IOBM_E_INVALID_ARG;
  if ((long long)g->nx * g->ny > 4096 || g->nz > 256) return IOBM_E_UNSUPPORTED;
  iobm_ctx ctx = new iobm_ctx_s();
  ctx->g.nx = g->nx; ctx->g.ny = g->ny; ctx->g.nz = g->nz; ctx->g.nf = g->nf;
  ctx->g.nxy = g->nx * g->ny;
  ctx->g.npts = (long long)ctx->g.nxy * g->nz;
  ctx->g.hx = g->hx; ctx->g.hy = g->hy; ctx->g.hz = g->hz;
  ctx->stream = (hipStream_t)stream;
  // central second-derivative weights (h = 1), orders 2, 4, 6
  static const double C[4][4] = {{0, 0, 0, 0},
                                 {-2.0, 1.0, 0, 0},
                                 {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0, 0},
                                 {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0}};
  for (int i = 0; i < 4; ++i) ctx->c[i] = C[g->nf][i];
  ctx->plan.x = make_plan1d(g->nx);
  ctx->plan.y = make_plan1d(g->ny);
  if (!plan_ok(ctx->plan.x) || !plan_ok(ctx->plan.y)) {
    delete ctx;
    return IOBM_E_UNSUPPORTED;
  }
  try {
    HIPCHK(hipGetDevice(&ctx->device));
    HIPCHK(hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    // the LDS kernels (readout, electrode term and plane FFT on non-square
    // planes) hold nf + 1 complex128 planes in one workgroup's LDS (gfx950:
    // 160 KiB per workgroup)
    const size_t max_lds = 160 * 1024;
    if ((size_t)(g->nf + 1) * ctx->g.nxy * sizeof(zd) > max_lds) {
      ctx->err = "nx*ny too large for the workgroup LDS at this FD order";
      throw Fail{IOBM_E_UNSUPPORTED};
    }
    {
      std::lock_guard<std::mutex> lock(static_ws_mu);
      if (ctx->device < 0 || ctx->device >= kMaxDevices) {
        ctx->err = "device index beyond the static workspace table";
        throw Fail{IOBM_E_UNSUPPORTED};
      }
      if (!static_ws_ptr[ctx->device]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        static_ws_ptr[ctx->device] = p;
      }
      ctx->static_ws = static_ws_ptr[ctx->device];
    }
    std::vector<zd> tx(g->nx), ty(g->ny);
    std::vector<zf> fx(g->nx), fy(g->ny);
    for (int k = 0; k < g->nx; ++k) {
      double a = -2.0 * M_PI * k / g->nx;
      tx[k] = mk(cos(a), sin(a));
      fx[k] = mk((float)cos(a), (float)sin(a));
    }
    for (int k = 0; k < g->ny; ++k) {
      double a = -2.0 * M_PI * k / g->ny;
      ty[k] = mk(cos(a), sin(a));
      fy[k] = mk((float)cos(a), (float)sin(a));
    }
    HIPCHK(hipMalloc(&ctx->twx_d, g->nx * sizeof(zd)));
    HIPCHK(hipMalloc(&ctx->twy_d, g->ny * sizeof(zd)));
    HIPCHK(hipMalloc(&ctx->twx_f, g->nx * sizeof(zf)));
    HIPCHK(hipMalloc(&ctx->twy_f, g->ny * sizeof(zf)));
    HIPCHK(hipMemcpy(ctx->twx_d, tx.data(), g->nx * sizeof(zd), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->twy_d, ty.data(), g->ny * sizeof(zd), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->twx_f, fx.data(), g->nx * sizeof(zf), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->twy_f, fy.data(), g->ny * sizeof(zf), hipMemcpyHostToDevice));
    {
      // the z filter's paired layout (zpair_mode): count the pairs and check
      // that they cover every lateral mode once, each non-self pair being
      // (k, -k); the layout stays off otherwise
      const int nx = g->nx, ny = g->ny, nxy = nx * ny;
      std::vector<char> seen(nxy, 0);
      int npair = 0, covered = 0;
      bool ok = true;
      for (;; ++npair) {
        bool s0 = false, s1 = false;
        const int a = zpair_mode(npair, 0, ny, nx, s0), b = zpair_mode(npair, 1, ny, nx, s1);
        if (a >= nxy) break;
        const int pa = ((ny - a / nx) % ny) * nx + (nx - a % nx) % nx;
        if (s0 ? pa != a : (b >= nxy || pa != b)) ok = false;
        for (int m : {a, b})
          if (m < nxy) {
            if (seen[m]) ok = false;
            seen[m] = 1;
            ++covered;
          }
      }
      ctx->zpair_nmb = ok && covered == nxy ? (npair + 31) / 32 : 0;
    }
    HIPCHK(hipMalloc(&ctx->arena_d, kRegion * kRegions));
    HIPCHK(hipHostMalloc(&ctx->arena_h, kRegion * kRegions, hipHostMallocDefault));
    HIPCHK(hipMalloc(&ctx->V_d, ctx->g.npts * sizeof(double)));
    HIPCHK(hipMalloc(&ctx->V_f, ctx->g.npts * sizeof(float)));
  } catch (Fail& f) {
    iobm_destroy(ctx);
    return f.s;
  }
  *out = ctx;
  return IOBM_OK;
}

iobm_status iobm_profile_begin(iobm_ctx ctx, int32_t class_mask) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (class_mask < 0 || class_mask >= (1 << (IOBM_K_BLOCH_VECTOR + 1)))
    return fail(ctx, IOBM_E_INVALID_ARG, "bad kernel class mask");
  ctx->prof_mask = class_mask;
  ctx->prof_used = 0;
  return IOBM_OK;
}

iobm_status iobm_profile_end(iobm_ctx ctx, int32_t kernel_class, int32_t* launches, double* total_ms,
                             double* alg_bytes) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(ctx, IOBM_E_DEVICE, hipGetErrorString(e));
  double ms = 0, bytes = 0;
  int n = 0;
  for (size_t k = 0; k < ctx->prof_used; ++k) {
    if (ctx->prof_cls[k] != kernel_class) continue;
    float t = 0;
    if (hipEventElapsedTime(&t, ctx->prof_ev[2 * k], ctx->prof_ev[2 * k + 1]) == hipSuccess) ms += t;
    bytes += ctx->prof_bytes[k];
    ++n;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (alg_bytes) *alg_bytes = bytes;
  return IOBM_OK;
}

iobm_status iobm_get_launch_shape(iobm_ctx ctx, int32_t precision, iobm_launch_shape* shape) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (!shape || (precision != IOBM_C128 && precision != IOBM_C64_REFINED))
    return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  *shape = launch_shape_in_effect(ctx, precision == IOBM_C128 ? 0 : 1);
  return IOBM_OK;
}

iobm_status iobm_set_launch_shape(iobm_ctx ctx, int32_t precision, const iobm_launch_shape* shape) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (precision != IOBM_C128 && precision != IOBM_C64_REFINED) return fail(ctx, IOBM_E_INVALID_ARG, "bad precision");
  const int p = precision == IOBM_C128 ? 0 : 1;
  if (!shape) {  // unpin: the next solve in this precision tunes again
    ctx->shape[p] = iobm_launch_shape{};
    ctx->tuned[p] = ctx->pinned[p] = false;
    return IOBM_OK;
  }
  std::string why;
  if (shape->stencil < 0 || shape->stencil > 2 || shape->plane_fft < 0 || shape->plane_fft > 2 ||
      shape->points_per_thread < 0 || shape->planes_per_block < 0 || shape->zfilter_chunk < 0 ||
      shape->rz_pass < 0 || shape->rz_pass > 2)
    return fail(ctx, IOBM_E_INVALID_ARG, "launch shape field out of range");
  if (!launch_shape_valid(ctx, p, *shape, why)) return fail(ctx, IOBM_E_UNSUPPORTED, why);
  ctx->shape[p] = *shape;
  ctx->tuned[p] = ctx->pinned[p] = true;
  return IOBM_OK;
}

iobm_status iobm_destroy(iobm_ctx ctx) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  for (hipEvent_t ev : ctx->prof_ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : ctx->cap_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  for (auto& e : ctx->pool)
    if (e.first) (void)hipFree(e.first);
  void* ptrs[] = {ctx->twx_d, ctx->twy_d, ctx->twx_f, ctx->twy_f, ctx->V_d, ctx->V_f, ctx->modes_d, ctx->sig_d,
                  ctx->sig_f, ctx->mode_flags_d, ctx->sdiag_d,
                  ctx->kb.uvox, ctx->kb.Bd, ctx->kb.Bf, ctx->kb.Btd, ctx->kb.Btf, ctx->kb.ctile, ctx->kb.prange,
                  ctx->kb.hD, ctx->kb.diag_d, ctx->arena_d};
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->arena_h) (void)hipHostFree(ctx->arena_h);
  if (ctx->rb_h) (void)hipHostFree(ctx->rb_h);
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete ctx;
  return IOBM_OK;
}

}  // extern "C"

namespace {
__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, long long n, int* bad) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double v = a[i];
    if (!isfinite(v)) bad[0] = 1;
    b[i] = (float)v;
  }
}
}  // namespace

extern "C" {

iobm_status iobm_set_potential(iobm_ctx ctx, const double* V, int32_t on_device) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (!V) return fail(ctx, IOBM_E_INVALID_ARG, "V is NULL");
  try {
    const long long n = ctx->g.npts;
    HIPCHK(hipMemcpyAsync(ctx->V_d, V, n * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
    int* bad = (int*)((char*)ctx->arena_d + 63 * kRegion);
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
    hipLaunchKernelGGL(k_to_float, dim3(256), dim3(256), 0, ctx->stream, ctx->V_d, ctx->V_f, n, bad);
    HIPCHK(hipGetLastError());
    int bad_h = 0;
    HIPCHK(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    if (bad_h) {
      ctx->have_V = false;
      return fail(ctx, IOBM_E_INVALID_ARG, "V contains a non-finite value");
    }
    ctx->have_V = true;
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_set_nonlocal(iobm_ctx ctx, int32_t ncen, int32_t rank, const int32_t* nsupport,
                              const int64_t* support_idx, const double* beta, const double* D) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  KBData& kb = ctx->kb;
  if (ncen < 0 || (ncen > 0 && (rank < 1 || rank > 8 || !nsupport || !support_idx || !beta || !D)))
    return fail(ctx, IOBM_E_INVALID_ARG, "bad nonlocal arguments");
  if (ncen * rank > 128) return fail(ctx, IOBM_E_UNSUPPORTED, "more than 128 projectors");
  // validate
  long long tot = 0;
  for (int a = 0; a < ncen; ++a) {
    if (nsupport[a] < 0) return fail(ctx, IOBM_E_INVALID_ARG, "negative support size");
    tot += nsupport[a];
  }
  for (long long i = 0; i < tot; ++i)
    if (support_idx[i] < 0 || support_idx[i] >= ctx->g.npts)
      return fail(ctx, IOBM_E_INVALID_ARG, "support index out of range");
  for (long long i = 0; i < tot * rank; ++i)
    if (!isfinite(beta[i])) return fail(ctx, IOBM_E_INVALID_ARG, "non-finite projector value");
  for (int a = 0; a < ncen; ++a)
    for (int p = 0; p < rank; ++p)
      for (int q = 0; q < rank; ++q) {
        double x = D[(a * rank + p) * rank + q], y = D[(a * rank + q) * rank + p];
        if (!isfinite(x)) return fail(ctx, IOBM_E_INVALID_ARG, "non-finite D");
        if (fabs(x - y) > 1e-12 * (fabs(x) + fabs(y) + 1e-300))
          return fail(ctx, IOBM_E_INVALID_ARG, "D must be symmetric (A must stay complex symmetric)");
      }
  // union of supports, dense projector matrix on it
  std::map<long long, int> uidx;
  {
    long long off = 0;
    for (int a = 0; a < ncen; ++a) {
      for (int k = 0; k < nsupport[a]; ++k) {
        long long v = support_idx[off + k];
        if (!uidx.count(v)) {
          int id = (int)uidx.size();
          uidx[v] = id;
        }
      }
      off += nsupport[a];
    }
  }
  // order the union by voxel id for coalesced gathers
  std::vector<int> uvox;
  uvox.reserve(uidx.size());
  {
    int id = 0;
    for (auto& kv : uidx) {
      kv.second = id++;
      uvox.push_back((int)kv.first);
    }
  }
  const int nproj = ncen * rank;
  const int npad = std::max(16, (nproj + 15) / 16 * 16);
  const int nu = (int)uvox.size();
  std::vector<double> Bm((size_t)nu * npad, 0.0);
  {
    long long off = 0, boff = 0;
    for (int a = 0; a < ncen; ++a) {
      for (int p = 0; p < rank; ++p)
        for (int k = 0; k < nsupport[a]; ++k) {
          int u = uidx[support_idx[off + k]];
          Bm[(size_t)u * npad + a * rank + p] += beta[boff + (long long)p * nsupport[a] + k];
        }
      off += nsupport[a];
      boff += (long long)rank * nsupport[a];
    }
  }
  const double h3 = ctx->g.hx * ctx->g.hy * ctx->g.hz;
  std::vector<double> hD((size_t)std::max(1, nproj * nproj), 0.0);
  for (int a = 0; a < ncen; ++a)
    for (int p = 0; p < rank; ++p)
      for (int q = 0; q < rank; ++q)
        hD[(size_t)(a * rank + p) * nproj + a * rank + q] = h3 * D[(a * rank + p) * rank + q];
  std::vector<float> Bf(Bm.begin(), Bm.end());
  std::vector<double> Bt((size_t)nu * nproj);
  for (int u = 0; u < nu; ++u)
    for (int p = 0; p < nproj; ++p) Bt[(size_t)p * nu + u] = Bm[(size_t)u * npad + p];
  std::vector<float> Btf(Bt.begin(), Bt.end());
  // where the projectors vanish: nonzero tiles per 64-voxel chunk of the
  // projection, nonzero projector range per 256-voxel block of the
  // back-projection
  std::vector<int> ctile((nu + 63) / 64, 0), prange(2 * (size_t)((nu + 255) / 256));
  for (size_t b = 0; b < prange.size() / 2; ++b) {
    prange[2 * b] = nproj;
    prange[2 * b + 1] = 0;
  }
  for (int u = 0; u < nu; ++u)
    for (int p = 0; p < nproj; ++p)
      if (Bm[(size_t)u * npad + p] != 0.0) {
        ctile[u / 64] |= 1 << (p / 16);
        int* r = &prange[2 * (size_t)(u / 256)];
        r[0] = std::min(r[0], p);
        r[1] = std::max(r[1], p + 1);
      }
  // diagonal of B h^3 D B^T per voxel (zero off the supports)
  std::vector<double> kdiag(nu > 0 ? (size_t)ctx->g.npts : 0, 0.0);
  for (int u = 0; u < nu; ++u) {
    double acc = 0;
    for (int p = 0; p < nproj; ++p)
      for (int q = 0; q < nproj; ++q) acc += Bm[(size_t)u * npad + p] * hD[(size_t)p * nproj + q] * Bm[(size_t)u * npad + q];
    kdiag[uvox[u]] = acc;
  }
  try {
    stream_sync(ctx);
    void* old[] = {kb.uvox, kb.Bd, kb.Bf, kb.Btd, kb.Btf, kb.ctile, kb.prange, kb.hD, kb.diag_d};
    for (void* p : old)
      if (p) (void)hipFree(p);
    kb = KBData();
    if (ncen == 0 || nu == 0) return IOBM_OK;
    HIPCHK(hipMalloc(&kb.uvox, nu * sizeof(int)));
    HIPCHK(hipMalloc(&kb.Bd, Bm.size() * sizeof(double)));
    HIPCHK(hipMalloc(&kb.Bf, Bf.size() * sizeof(float)));
    HIPCHK(hipMalloc(&kb.Btd, Bt.size() * sizeof(double)));
    HIPCHK(hipMalloc(&kb.Btf, Btf.size() * sizeof(float)));
    HIPCHK(hipMalloc(&kb.ctile, ctile.size() * sizeof(int)));
    HIPCHK(hipMalloc(&kb.prange, prange.size() * sizeof(int)));
    HIPCHK(hipMalloc(&kb.hD, hD.size() * sizeof(double)));
    HIPCHK(hipMemcpy(kb.uvox, uvox.data(), nu * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(kb.Bd, Bm.data(), Bm.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(kb.Bf, Bf.data(), Bf.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(kb.Btd, Bt.data(), Bt.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(kb.Btf, Btf.data(), Btf.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(kb.ctile, ctile.data(), ctile.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(kb.prange, prange.data(), prange.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(kb.hD, hD.data(), hD.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&kb.diag_d, kdiag.size() * sizeof(double)));
    HIPCHK(hipMemcpy(kb.diag_d, kdiag.data(), kdiag.size() * sizeof(double), hipMemcpyHostToDevice));
    kb.ncen = ncen;
    kb.rank = rank;
    kb.nproj = nproj;
    kb.nproj_pad = npad;
    kb.nu = nu;
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_channels(iobm_ctx ctx, double E, int32_t* nopen, int32_t* ids, double* kz, double* v) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (!nopen || !isfinite(E)) return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  try {
    ensure_modes(ctx, std::vector<double>{E});
    int n = 0;
    for (int m = 0; m < ctx->g.nxy; ++m) {
      const ModeData& md = host_modes(ctx)[m];
      if (!(md.flags & MODE_OPEN)) continue;
      if (ids) ids[n] = m;
      if (kz) kz[n] = atan2(md.xp.im, md.xp.re) / ctx->g.hz;
      if (v) v[n] = md.v;
      ++n;
    }
    *nopen = n;
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_self_energy(iobm_ctx ctx, double E, double* sigma) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (!sigma || !isfinite(E)) return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  try {
    ensure_modes(ctx, std::vector<double>{E});
    const int nf = ctx->g.nf;
    for (int m = 0; m < ctx->g.nxy; ++m)
      for (int i = 0; i < nf * nf; ++i) {
        sigma[2 * ((size_t)m * nf * nf + i)] = host_modes(ctx)[m].sig[i].re;
        sigma[2 * ((size_t)m * nf * nf + i) + 1] = host_modes(ctx)[m].sig[i].im;
      }
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_apply(iobm_ctx ctx, double E, int32_t nrhs, const void* x, void* y, int32_t precision) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (nrhs < 0 || (nrhs > 0 && (!x || !y)) || !isfinite(E) ||
      (precision != IOBM_C128 && precision != IOBM_C64_REFINED))
    return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  if (!ctx->have_V) return fail(ctx, IOBM_E_BAD_STATE, "iobm_set_potential has not been called");
  if (x == y) return fail(ctx, IOBM_E_INVALID_ARG, "x and y must not overlap");
  if (nrhs == 0) return IOBM_OK;
  try {
    ensure_modes(ctx, std::vector<double>{E});
    std::vector<int> e(nrhs, 0);
    std::vector<double> Ev(nrhs, E);
    int* e_d = upload(ctx, S_IDX, e, 0);
    double* E_d = upload(ctx, S_IDX, Ev, 32 * 1024);
    if (ctx->kb.ncen > 0) (void)kb_scratch(ctx, kb_proj_bytes(ctx, nrhs));
    if (precision == IOBM_C128)
      HIPCHK(launch_apply<double>(ctx, (const zd*)x, (zd*)y, nrhs, E_d, e_d, ctx->modes_d, nullptr));
    else
      HIPCHK(launch_apply<float>(ctx, (const zf*)x, (zf*)y, nrhs, E_d, e_d, ctx->modes_d, nullptr));
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_precondition(iobm_ctx ctx, int32_t precond, double alpha, double E, int32_t nrhs,
                              const void* r, void* z, int32_t precision, double* rz) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (nrhs < 0 || (nrhs > 0 && (!r || !z)) || !isfinite(E) || !(alpha > 0) ||
      (precision != IOBM_C128 && precision != IOBM_C64_REFINED) || precond < 0 || precond > IOBM_PC_JACOBI)
    return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  if (r == z) return fail(ctx, IOBM_E_INVALID_ARG, "r and z must not overlap");
  if (nrhs == 0) return IOBM_OK;
  try {
    const long long vol = ctx->g.npts;
    const int slots = precond_slots(ctx, precond);
    Partial* part = rz ? (Partial*)workspace(ctx, S_PARTZ, (size_t)nrhs * slots * sizeof(Partial)) : nullptr;
    if (precond == IOBM_PC_NONE) {
      size_t es = precision == IOBM_C128 ? sizeof(zd) : sizeof(zf);
      HIPCHK(hipMemcpyAsync(z, r, (size_t)nrhs * vol * es, hipMemcpyDeviceToDevice, ctx->stream));
      if (part && precision == IOBM_C128) HIPCHK(launch_dot<double>(ctx, (const zd*)r, (const zd*)r, nrhs, nullptr, part));
      if (part && precision != IOBM_C128) HIPCHK(launch_dot<float>(ctx, (const zf*)r, (const zf*)r, nrhs, nullptr, part));
    } else if (precond == IOBM_PC_TRUNCATED_LAPLACIAN) {
      if (precision == IOBM_C128)
        HIPCHK(launch_precond_laplacian<double>(ctx, alpha, (const zd*)r, (zd*)z, nrhs, nullptr, part));
      else
        HIPCHK(launch_precond_laplacian<float>(ctx, alpha, (const zf*)r, (zf*)z, nrhs, nullptr, part));
    } else if (precond == IOBM_PC_JACOBI) {
      ensure_modes(ctx, std::vector<double>{E});
      std::vector<int> e(nrhs, 0);
      std::vector<double> Ev(nrhs, E);
      int* e_d = upload(ctx, S_IDX, e, 0);
      double* E_d = upload(ctx, S_IDX, Ev, 32 * 1024);
      if (precision == IOBM_C128)
        HIPCHK(launch_precond_jacobi<double>(ctx, (const zd*)r, (zd*)z, nrhs, e_d, E_d, nullptr, part));
      else
        HIPCHK(launch_precond_jacobi<float>(ctx, (const zf*)r, (zf*)z, nrhs, e_d, E_d, nullptr, part));
    } else {
      ensure_modes(ctx, std::vector<double>{E});
      std::vector<int> e(nrhs, 0);
      int* e_d = upload(ctx, S_IDX, e, 0);
      if (precision == IOBM_C128) {
        zd* pf = (zd*)workspace(ctx, S_PF, (size_t)nrhs * vol * sizeof(zd));
        HIPCHK(launch_precond_fft<double>(ctx, (const zd*)r, (zd*)z, pf, nrhs, e_d, ctx->modes_d, nullptr, part));
      } else {
        zf* pf = (zf*)workspace(ctx, S_PF, (size_t)nrhs * vol * sizeof(zf));
        HIPCHK(launch_precond_fft<float>(ctx, (const zf*)r, (zf*)z, pf, nrhs, e_d, ctx->modes_d, nullptr, part));
      }
    }
    if (rz) {
      // the partials, summed per vector in slot order as the solver does
      std::vector<Partial> h((size_t)nrhs * slots);
      HIPCHK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(Partial), hipMemcpyDeviceToHost, ctx->stream));
      stream_sync(ctx);
      for (int i = 0; i < nrhs; ++i) {
        double re = 0, im = 0;
        for (int k = 0; k < slots; ++k) { re += h[(size_t)i * slots + k].re; im += h[(size_t)i * slots + k].im; }
        rz[2 * i] = re;
        rz[2 * i + 1] = im;
      }
    }
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_rhs(iobm_ctx ctx, double E, int32_t n, const int32_t* ids, int32_t side, void* b) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!ids || !b)) || !isfinite(E) || (side != 0 && side != 1))
    return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  if (n == 0) return IOBM_OK;
  try {
    ensure_modes(ctx, std::vector<double>{E});
    for (int k = 0; k < n; ++k)
      if (ids[k] < 0 || ids[k] >= ctx->g.nxy || !(ctx->mode_flags_h[ids[k]] & MODE_OPEN))
        return fail(ctx, IOBM_E_INVALID_ARG, "channel not open");
    std::vector<int> e(n, 0), m(ids, ids + n), kind(n, 0);
    int* e_d = upload(ctx, S_IDX, e, 0);
    int* m_d = upload(ctx, S_IDX, m, 16 * 1024);
    int* k_d = upload(ctx, S_IDX, kind, 32 * 1024);
    HIPCHK(launch_rhs(ctx, n, e_d, m_d, k_d, side, ctx->modes_d, (zd*)b, false));
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_solve(iobm_ctx ctx, const iobm_solve_opts* opts, int32_t nE, const double* E,
                       const int32_t* ninc, const int32_t* inc, void* psi, double* t, double* T, double* R,
                       iobm_solve_stat* st) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  try {
    validate_opts(ctx, opts);
    if (nE < 0 || (nE > 0 && (!E || !ninc))) return fail(ctx, IOBM_E_INVALID_ARG, "bad energy list");
    if (!ctx->have_V) return fail(ctx, IOBM_E_BAD_STATE, "iobm_set_potential has not been called");
    int ninc_total = 0;
    for (int e = 0; e < nE; ++e) {
      if (!isfinite(E[e])) return fail(ctx, IOBM_E_INVALID_ARG, "non-finite energy");
      if (ninc[e] > 0) ninc_total += ninc[e];
    }
    if (ninc_total > 0 && !inc) return fail(ctx, IOBM_E_INVALID_ARG, "inc is NULL");
    if (nE == 0) return IOBM_OK;
    const iobm_solve_opts& o = *opts;
    ensure_modes(ctx, std::vector<double>(E, E + nE), true);
    SolveRun run;
    run_solve(ctx, o, nE, E, ninc, inc, run);
    const int nreq = (int)run.Q.e.size();
    const int nxy = ctx->g.nxy;
    if (psi) HIPCHK(launch_combine_psi<double>(ctx, nreq, run.x, (zd*)psi, run.qc, run.qs, run.qg));
    std::vector<double> TRh(2 * nreq);
    HIPCHK(hipMemcpyAsync(TRh.data(), run.TR, 2 * nreq * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    std::vector<zd> th;
    if (t) {
      th.resize((size_t)nreq * nxy);
      HIPCHK(hipMemcpyAsync(th.data(), run.t_out, th.size() * sizeof(zd), hipMemcpyDeviceToHost, ctx->stream));
    }
    stream_sync(ctx);
    if (T) for (int c = 0; c < nreq; ++c) T[c] = TRh[c];
    if (R) for (int c = 0; c < nreq; ++c) R[c] = TRh[nreq + c];
    if (t) {
      // per energy: [nopen(E)][ninc_e]
      size_t off = 0;
      int c0 = 0;
      for (int e = 0; e < nE; ++e) {
        int c1 = c0;
        while (c1 < nreq && run.Q.e[c1] == e) ++c1;
        const int* fl = &ctx->mode_flags_h[(size_t)e * nxy];
        int row = 0;
        for (int nu = 0; nu < nxy; ++nu) {
          if (!(fl[nu] & MODE_OPEN)) continue;
          for (int c = c0; c < c1; ++c) {
            zd v = th[(size_t)c * nxy + nu];
            t[2 * (off + (size_t)row * (c1 - c0) + (c - c0))] = v.re;
            t[2 * (off + (size_t)row * (c1 - c0) + (c - c0)) + 1] = v.im;
          }
          ++row;
        }
        off += (size_t)row * (c1 - c0);
        c0 = c1;
      }
    }
    const iobm_status worst = request_stats(run, TRh, st);
    if (worst != IOBM_OK) {
      ctx->err = "some right-hand sides did not converge";
      return worst;
    }
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_smatrix(iobm_ctx ctx, const iobm_solve_opts* opts, int32_t nE, const double* E, double* S,
                         iobm_solve_stat* st) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  try {
    validate_opts(ctx, opts);
    if (nE < 0 || (nE > 0 && (!E || !S))) return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
    if (!ctx->have_V) return fail(ctx, IOBM_E_BAD_STATE, "iobm_set_potential has not been called");
    for (int e = 0; e < nE; ++e)
      if (!isfinite(E[e])) return fail(ctx, IOBM_E_INVALID_ARG, "non-finite energy");
    if (nE == 0) return IOBM_OK;
    ensure_modes(ctx, std::vector<double>(E, E + nE), true);
    const int nxy = ctx->g.nxy, nf = ctx->g.nf;
    const ModeData* md = host_modes(ctx);
    // open channels per energy (ascending ids) and the offsets of S
    std::vector<std::vector<int>> open(nE);
    std::vector<size_t> soff(nE + 1, 0);
    int nstates = 0;
    for (int e = 0; e < nE; ++e) {
      for (int m = 0; m < nxy; ++m)
        if (ctx->mode_flags_h[(size_t)e * nxy + m] & MODE_OPEN) open[e].push_back(m);
      const size_t n = open[e].size();
      soff[e + 1] = soff[e] + 4 * n * n;
      nstates += (int)n;
    }
    std::vector<int> ninc(nE, -1);
    iobm_status worst = IOBM_OK;
    for (int side = 0; side < 2; ++side) {
      iobm_solve_opts o = *opts;
      o.side = side;
      SolveRun run;
      run_solve(ctx, o, nE, E, ninc.data(), nullptr, run);
      const int nreq = (int)run.Q.e.size();
      std::vector<zd> th((size_t)nreq * nxy), rh((size_t)nreq * nxy);
      std::vector<double> TRh(2 * nreq);
      HIPCHK(hipMemcpyAsync(th.data(), run.t_out, th.size() * sizeof(zd), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipMemcpyAsync(rh.data(), run.r_out, rh.size() * sizeof(zd), hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipMemcpyAsync(TRh.data(), run.TR, 2 * nreq * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      stream_sync(ctx);
      const iobm_status w = request_stats(run, TRh, st ? st + (size_t)side * nstates : nullptr);
      if (w != IOBM_OK) worst = w;
      // column block a = side; row block b = the lead of the outgoing wave.
      // Transmitted amplitudes come referred to the nf-th plane from the far
      // lead; the propagating wave gains x^(nf-1) up to the plane next to it.
      for (int c = 0; c < nreq; ++c) {
        const int e = run.Q.e[c], mu = run.Q.mode[c];
        const std::vector<int>& ids = open[e];
        const int n = (int)ids.size();
        const int j = (int)(std::lower_bound(ids.begin(), ids.end(), mu) - ids.begin());
        const ModeData* me = md + (size_t)e * nxy;
        for (int i = 0; i < n; ++i) {
          const int nu = ids[i];
          const double w_ = sqrt(me[nu].v / me[mu].v);
          zd tr = th[(size_t)c * nxy + nu];
          for (int k = 0; k < nf - 1; ++k) tr = tr * me[nu].xp;
          const zd rf = rh[(size_t)c * nxy + nu];
          const int col = side * n + j;
          const int row_r = side * n + i, row_t = (1 - side) * n + i;
          double* Se = S + 2 * soff[e];
          Se[2 * ((size_t)row_r * 2 * n + col)] = w_ * rf.re;
          Se[2 * ((size_t)row_r * 2 * n + col) + 1] = w_ * rf.im;
          Se[2 * ((size_t)row_t * 2 * n + col)] = w_ * tr.re;
          Se[2 * ((size_t)row_t * 2 * n + col) + 1] = w_ * tr.im;
        }
      }
    }
    if (worst != IOBM_OK) {
      ctx->err = "some right-hand sides did not converge";
      return worst;
    }
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_channels_bloch(iobm_ctx ctx, double E, double kx, double ky, int32_t* nopen, int32_t* ids,
                                double* kz, double* v) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (!nopen || !isfinite(E) || !isfinite(kx) || !isfinite(ky)) return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  try {
    ensure_modes(ctx, std::vector<double>{E}, false, std::vector<double>{kx * ctx->g.hx, ky * ctx->g.hy});
    int n = 0;
    for (int m = 0; m < ctx->g.nxy; ++m) {
      const ModeData& md = host_modes(ctx)[m];
      if (!(md.flags & MODE_OPEN)) continue;
      if (ids) ids[n] = m;
      if (kz) kz[n] = atan2(md.xp.im, md.xp.re) / ctx->g.hz;
      if (v) v[n] = md.v;
      ++n;
    }
    *nopen = n;
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

iobm_status iobm_smatrix_bloch(iobm_ctx ctx, const iobm_solve_opts* opts, double kx, double ky, int32_t nE,
                               const double* E, double* S_plus, double* S_minus, iobm_solve_stat* st) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  try {
    validate_opts(ctx, opts);
    if (nE < 0 || (nE > 0 && (!E || !S_plus || !S_minus)) || !isfinite(kx) || !isfinite(ky))
      return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
    if (opts->block != 0) return fail(ctx, IOBM_E_UNSUPPORTED, "the lateral-Bloch-vector solve has no block COCG");
    if (ctx->kb.ncen > 0)
      return fail(ctx, IOBM_E_UNSUPPORTED, "the lateral-Bloch-vector solve does not take a nonlocal term");
    if (!ctx->have_V) return fail(ctx, IOBM_E_BAD_STATE, "iobm_set_potential has not been called");
    for (int e = 0; e < nE; ++e)
      if (!isfinite(E[e])) return fail(ctx, IOBM_E_INVALID_ARG, "non-finite energy");
    if (nE == 0) return IOBM_OK;
    const GridDev& g = ctx->g;
    const int nxy = g.nxy, nf = g.nf;
    // mode table: entries 0..nE-1 at +kappa, nE..2nE-1 at -kappa
    std::vector<double> E2(E, E + nE), K2;
    E2.insert(E2.end(), E, E + nE);
    for (int e = 0; e < nE; ++e) { K2.push_back(kx * g.hx); K2.push_back(ky * g.hy); }
    for (int e = 0; e < nE; ++e) { K2.push_back(-kx * g.hx); K2.push_back(-ky * g.hy); }
    ensure_modes(ctx, E2, true, K2);
    const ModeData* md = host_modes(ctx);
    std::vector<std::vector<int>> openp(nE), openm(nE);
    std::vector<size_t> soff(nE + 1, 0);
    int nstates = 0;
    for (int e = 0; e < nE; ++e) {
      for (int m = 0; m < nxy; ++m) {
        if (ctx->mode_flags_h[(size_t)e * nxy + m] & MODE_OPEN) openp[e].push_back(m);
        if (ctx->mode_flags_h[(size_t)(nE + e) * nxy + m] & MODE_OPEN) openm[e].push_back(m);
      }
      if (openp[e].size() != openm[e].size()) {
        ctx->err = "open channels at +kappa and -kappa differ";
        throw Fail{IOBM_E_DEVICE};
      }
      const size_t n = openp[e].size();
      soff[e + 1] = soff[e] + 4 * n * n;
      nstates += (int)n;
    }
    BlochPhase ph;
    for (int n = 0; n < 4; ++n) {
      ph.x[n] = mk(cos(n * kx * g.hx), sin(n * kx * g.hx));
      ph.y[n] = mk(cos(n * ky * g.hy), sin(n * ky * g.hy));
    }
    const long long vol = g.npts;
    iobm_status worst = IOBM_OK;
    for (int side = 0; side < 2; ++side) {
      PairBatch B;
      for (int e = 0; e < nE; ++e)
        for (int mu : openp[e]) {
          const int mneg = neg_mode(g, mu);
          if (!std::binary_search(openm[e].begin(), openm[e].end(), mneg)) {
            ctx->err = "the partner channel at -kappa is closed";
            throw Fail{IOBM_E_DEVICE};
          }
          B.e.push_back(e); B.E.push_back(E[e]); B.mode.push_back(mu); B.sgn.push_back(1);
          B.e.push_back(nE + e); B.E.push_back(E[e]); B.mode.push_back(mneg); B.sgn.push_back(-1);
        }
      B.n = (int)B.e.size();
      if (B.n == 0) continue;
      zd* b = (zd*)workspace(ctx, S_B, (size_t)B.n * vol * sizeof(zd));
      zd* x = (zd*)workspace(ctx, S_XHI, (size_t)B.n * vol * sizeof(zd));
      {  // plane-wave right-hand sides in the gauge u (Eq. (6) at G + kappa)
        int* e_d = upload(ctx, S_IDX, B.e, 0);
        int* m_d = upload(ctx, S_IDX, B.mode, 16 * 1024);
        std::vector<int> kind(B.n, 0);
        int* k_d = upload(ctx, S_IDX, kind, 32 * 1024);
        HIPCHK(launch_rhs(ctx, B.n, e_d, m_d, k_d, side, ctx->modes_d, b, false));
      }
      SolveOut so;
      if (opts->precision == IOBM_C64_REFINED) solve_pair_batch<float>(ctx, *opts, ph, B, b, x, so);
      else solve_pair_batch<double>(ctx, *opts, ph, B, b, x, so);
      zd* amp = (zd*)workspace(ctx, S_AMP, (size_t)2 * B.n * nxy * sizeof(zd));
      int* e_d = upload(ctx, S_IDX, B.e, 0);
      HIPCHK(launch_readout(ctx, B.n, side, x, ctx->modes_d, e_d, amp, amp + (size_t)B.n * nxy));
      std::vector<zd> ah((size_t)2 * B.n * nxy);
      HIPCHK(hipMemcpyAsync(ah.data(), amp, ah.size() * sizeof(zd), hipMemcpyDeviceToHost, ctx->stream));
      stream_sync(ctx);
      const zd* an = ah.data();
      const zd* af = ah.data() + (size_t)B.n * nxy;
      // column a = side of the incident channel; row blocks: the lead of the
      // outgoing wave.  Amplitudes are referred to the plane next to their
      // lead (the transmitted wave gains x^(nf-1) from the nf-th plane).
      int pos = 0;
      for (int e = 0; e < nE; ++e) {
        const int n = (int)openp[e].size();
        for (int jj = 0; jj < n; ++jj, pos += 2) {
          for (int h = 0; h < 2; ++h) {
            const int slot = pos + h;
            const std::vector<int>& ids = h ? openm[e] : openp[e];
            const int mu = B.mode[slot];
            const int j = (int)(std::lower_bound(ids.begin(), ids.end(), mu) - ids.begin());
            const ModeData* me = md + (size_t)B.e[slot] * nxy;
            double* Se = (h ? S_minus : S_plus) + 2 * soff[e];
            for (int i = 0; i < n; ++i) {
              const int nu = ids[i];
              const double w_ = sqrt(me[nu].v / me[mu].v);
              zd tr = af[(size_t)slot * nxy + nu];
              for (int k = 0; k < nf - 1; ++k) tr = tr * me[nu].xp;
              zd rf = an[(size_t)slot * nxy + nu];
              if (nu == mu) rf = rf - me[mu].kin;
              const int col = side * n + j;
              const int row_r = side * n + i, row_t = (1 - side) * n + i;
              Se[2 * ((size_t)row_r * 2 * n + col)] = w_ * rf.re;
              Se[2 * ((size_t)row_r * 2 * n + col) + 1] = w_ * rf.im;
              Se[2 * ((size_t)row_t * 2 * n + col)] = w_ * tr.re;
              Se[2 * ((size_t)row_t * 2 * n + col) + 1] = w_ * tr.im;
            }
            if (so.status[slot] != IOBM_OK) worst = (iobm_status)so.status[slot];
          }
          if (st) {  // per pair: [side][sum_e n_e]
            iobm_solve_stat& q = st[(size_t)side * nstates + pos / 2];
            q.iters = so.iters[pos];
            q.refinements = so.refin[pos];
            q.status = so.status[pos] != IOBM_OK ? so.status[pos] : so.status[pos + 1];
            q.pad_ = 0;
            q.rel_residual = std::max(so.rel[pos], so.rel[pos + 1]);
            q.flux_error = 0.0;
          }
        }
      }
    }
    if (st) {  // flux error of the +kappa column: sum_b |S[b nu][a mu]|^2 - 1
      int pos = 0;
      for (int e = 0; e < nE; ++e) {
        const int n = (int)openp[e].size();
        const double* Se = S_plus + 2 * soff[e];
        for (int side = 0; side < 2; ++side)
          for (int j = 0; j < n; ++j) {
            double f = 0;
            for (int i = 0; i < 2 * n; ++i) {
              const double re = Se[2 * ((size_t)i * 2 * n + side * n + j)];
              const double im = Se[2 * ((size_t)i * 2 * n + side * n + j) + 1];
              f += re * re + im * im;
            }
            st[(size_t)side * nstates + pos + j].flux_error = f - 1.0;
          }
        pos += n;
      }
    }
    if (worst != IOBM_OK) {
      ctx->err = "some scattering states did not converge";
      return worst;
    }
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

}  // extern "C"

extern "C" iobm_status iobm_grad_transmission(iobm_ctx ctx, const iobm_solve_opts* opts, int32_t nE,
                                              const double* E, double* T_total, void* dT_dV) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  try {
    validate_opts(ctx, opts);
    if (nE < 1 || !E || !T_total || !dT_dV) return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
    if (!ctx->have_V) return fail(ctx, IOBM_E_BAD_STATE, "iobm_set_potential has not been called");
    for (int e = 0; e < nE; ++e)
      if (!isfinite(E[e])) return fail(ctx, IOBM_E_INVALID_ARG, "non-finite energy");
    const iobm_solve_opts& o = *opts;
    ensure_modes(ctx, std::vector<double>(E, E + nE), true);
    std::vector<int> ninc(nE, -1);
    Batch B;
    Request Q;
    plan_requests(ctx, nE, E, ninc.data(), nullptr, B, Q);
    const int nb = B.n, nreq = (int)Q.e.size();
    const long long vol = ctx->g.npts;
    const int nxy = ctx->g.nxy;
    *T_total = 0.0;
    HIPCHK(hipMemsetAsync(dT_dV, 0, (size_t)vol * sizeof(double), ctx->stream));
    if (nb == 0) {
      stream_sync(ctx);
      return IOBM_OK;
    }
    // the forward solves A u_b = rhs_b (slots 0 .. nb-1) and the adjoint
    // solves A w_b = l_b in the same real lateral basis (slots nb .. 2nb-1):
    // the adjoint right-hand sides do not depend on u, so both run in one
    // batch and share every iteration
    zd* b = (zd*)workspace(ctx, S_B, (size_t)2 * nb * vol * sizeof(zd));
    zd* u = (zd*)workspace(ctx, S_XHI, (size_t)2 * nb * vol * sizeof(zd));
    zd* w = u + (size_t)nb * vol;
    {
      int* e_d = upload(ctx, S_IDX, B.e, 0);
      int* m_d = upload(ctx, S_IDX, B.mode, 16 * 1024);
      int* k_d = upload(ctx, S_IDX, B.kind, 32 * 1024);
      HIPCHK(launch_rhs(ctx, nb, e_d, m_d, k_d, o.side, ctx->modes_d, b, true));
      HIPCHK(launch_rhs_adjoint(ctx, nb, e_d, m_d, k_d, o.side, ctx->modes_d, b + (size_t)nb * vol));
    }
    Batch B2 = B;
    B2.n = 2 * nb;
    B2.e.insert(B2.e.end(), B.e.begin(), B.e.end());
    B2.E.insert(B2.E.end(), B.E.begin(), B.E.end());
    B2.mode.insert(B2.mode.end(), B.mode.begin(), B.mode.end());
    B2.kind.insert(B2.kind.end(), B.kind.begin(), B.kind.end());
    SolveOut s2;
    solve_batch(ctx, o, B2, b, u, s2);
    zd* amp = (zd*)workspace(ctx, S_AMP, (size_t)(2 * nb + 2 * nreq) * nxy * sizeof(zd));
    zd* amp_near = amp;
    zd* amp_far = amp + (size_t)nb * nxy;
    zd* t_out = amp + (size_t)2 * nb * nxy;
    zd* r_out = t_out + (size_t)nreq * nxy;
    double* TR = (double*)workspace(ctx, S_TR, (size_t)2 * nreq * sizeof(double) + 64);
    int* e_d = upload(ctx, S_IDX, B.e, 0);
    HIPCHK(launch_readout(ctx, nb, o.side, u, ctx->modes_d, e_d, amp_near, amp_far));
    int* qe = upload(ctx, S_IDX, Q.e, 16 * 1024);
    int* qm = upload(ctx, S_IDX, Q.mode, 24 * 1024);
    int* qc = upload(ctx, S_IDX, Q.c, 32 * 1024);
    int* qs = upload(ctx, S_IDX, Q.s, 40 * 1024);
    int* qg = upload(ctx, S_IDX, Q.sgn, 48 * 1024);
    HIPCHK(launch_combine(ctx, nreq, qe, qm, qc, qs, qg, ctx->modes_d, amp_near, amp_far, t_out, r_out, TR,
                          TR + nreq));
    std::vector<double> TRh(2 * nreq);
    HIPCHK(hipMemcpyAsync(TRh.data(), TR, 2 * nreq * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    double Ttot = 0;
    for (int c = 0; c < nreq; ++c) Ttot += TRh[c];
    // D blocks per energy and the gradient contraction
    std::vector<int> base(nE + 1, 0);
    for (int k = 0; k < nb; ++k) base[B.e[k] + 1]++;
    for (int e = 0; e < nE; ++e) base[e + 1] += base[e];
    std::vector<long long> dbase(nE, 0);
    long long dtot = 0;
    int nmax = 0;
    for (int e = 0; e < nE; ++e) {
      int n = base[e + 1] - base[e];
      dbase[e] = dtot;
      dtot += (long long)n * n;
      nmax = std::max(nmax, n);
    }
    std::vector<int> chan(2 * nb, -1);
    std::vector<zd> pc(2 * nb, mk(0.0, 0.0)), qc2(2 * nb, mk(0.0, 0.0));
    auto add = [&](int k, int c, zd p, zd q) {
      int s = chan[2 * k] < 0 ? 0 : 1;
      chan[2 * k + s] = c;
      pc[2 * k + s] = p;
      qc2[2 * k + s] = q;
    };
    for (int c = 0; c < nreq; ++c) {
      add(Q.c[c], c, mk(1.0, 0.0), mk(1.0, 0.0));
      if (Q.s[c] >= 0) {
        double sg = (double)Q.sgn[c];
        add(Q.s[c], c, mk(0.0, sg), mk(0.0, -sg));
      }
    }
    zd* Dd = (zd*)workspace(ctx, S_GRAD_D, (size_t)std::max<long long>(1, dtot) * sizeof(zd));
    int* base_d = upload(ctx, S_IDX, base, 64 * 1024);
    long long* dbase_d = upload(ctx, S_IDX, dbase, 72 * 1024);
    int* chan_d = upload(ctx, S_IDX, chan, 80 * 1024);
    zd* pc_d = upload(ctx, S_IDX, pc, 96 * 1024);
    zd* qc_d = upload(ctx, S_IDX, qc2, 160 * 1024);
    int* qm2 = upload(ctx, S_IDX, Q.mode, 168 * 1024);
    int* qe2 = upload(ctx, S_IDX, Q.e, 176 * 1024);
    HIPCHK(launch_grad_D(ctx, nE, nmax, base_d, chan_d, pc_d, qc_d, qm2, qe2, ctx->modes_d, t_out, Dd, dbase_d));
    HIPCHK(launch_grad(ctx, nE, base_d, dbase_d, Dd, u, w, (double*)dT_dV));
    stream_sync(ctx);
    *T_total = Ttot;
    for (int k = 0; k < 2 * nb; ++k)
      if (s2.status[k] != IOBM_OK) {
        ctx->err = k < nb ? "forward solve did not converge" : "adjoint solve did not converge";
        return (iobm_status)s2.status[k];
      }
  } catch (Fail& f) {
    return f.s;
  }
  return IOBM_OK;
}

// ============================================== allocation-free preconditioner
namespace {

// OR of the mode flags of one energy's table (one block, fixed order).
__global__ void __launch_bounds__(256) k_mode_flags_or(const ModeData* __restrict__ modes, int n, int* out) {
  __shared__ int sh[256];
  int f = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) f |= modes[i].flags;
  sh[threadIdx.x] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) a |= sh[i];
    out[0] = a;
  }
}

// Sum of each vector's partials of r^T z in slot order (the order the host
// sum of iobm_precondition takes), one thread per vector.
__global__ void k_sum_partials(const Partial* __restrict__ part, int nrhs, int slots, double* __restrict__ rz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrhs) return;
  double re = 0, im = 0;
  for (int k = 0; k < slots; ++k) {
    re += part[(long long)i * slots + k].re;
    im += part[(long long)i * slots + k].im;
  }
  rz[2 * i] = re;
  rz[2 * i + 1] = im;
}

// Zero fill (a kernel rather than a memset node, for callers that capture).
__global__ void k_fill_zero(unsigned long long* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Host-to-device copy of a small array through the pinned arena (region r),
// without building a host vector.
void* upload_bytes(iobm_ctx ctx, int region, const void* src, size_t bytes) {
  if (ctx->region_pending[region]) stream_sync(ctx);
  char* h = (char*)ctx->arena_h + (size_t)region * kRegion;
  char* d = (char*)ctx->arena_d + (size_t)region * kRegion;
  memcpy(h, src, bytes);
  HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, ctx->stream));
  ctx->region_pending[region] = 1;
  return d;
}

template <typename T>
void precondition_static(iobm_ctx ctx, int precond, double alpha, double E, int nrhs, const void* r, void* z,
                         double* rz) {
  const long long vol = ctx->g.npts;
  const int nxy = ctx->g.nxy;
  const int slots = precond_slots(ctx, precond);
  // layout of the static workspace: mode table and flag word (lateral-Fourier
  // preconditioner), plane-FFT scratch, partials, per-vector r^T z
  size_t off = 0;
  const size_t o_modes = off;
  if (precond == IOBM_PC_LATERAL_FFT) off += align256((size_t)nxy * sizeof(ModeData)) + 256;
  const size_t o_pf = off;
  if (precond == IOBM_PC_LATERAL_FFT) off += align256((size_t)nrhs * vol * sizeof(cplx<T>));
  const size_t o_part = off;
  if (rz) off += align256((size_t)nrhs * slots * sizeof(Partial)) + align256((size_t)nrhs * 2 * sizeof(double));
  if (off > IOBM_STATIC_WS_BYTES || (rz && (size_t)nrhs * 2 * sizeof(double) > kRegion) ||
      (size_t)nrhs * sizeof(int) > kRegion) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "iobm_precondition_noalloc needs %zu bytes of workspace for %d vectors; the static workspace holds %llu",
             off, nrhs, (unsigned long long)IOBM_STATIC_WS_BYTES);
    ctx->err = buf;
    throw Fail{IOBM_E_UNSUPPORTED};
  }
  char* ws = (char*)ctx->static_ws;
  Partial* part = rz ? (Partial*)(ws + o_part) : nullptr;
  double* rz_d = rz ? (double*)(ws + o_part + align256((size_t)nrhs * slots * sizeof(Partial))) : nullptr;
  if (part) {  // every slot is written by its block; cleared so that no stale value can survive
    const long long n8 = (long long)nrhs * slots * sizeof(Partial) / 8;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<long long>(1024, (n8 + 255) / 256)), dim3(256), 0,
                       ctx->stream, (unsigned long long*)part, n8);
    HIPCHK(hipGetLastError());
  }
  if (precond == IOBM_PC_NONE) {
    HIPCHK(hipMemcpyAsync(z, r, (size_t)nrhs * vol * sizeof(cplx<T>), hipMemcpyDeviceToDevice, ctx->stream));
    if (part) HIPCHK(launch_dot<T>(ctx, (const cplx<T>*)r, (const cplx<T>*)r, nrhs, nullptr, part));
  } else if (precond == IOBM_PC_TRUNCATED_LAPLACIAN) {
    HIPCHK(launch_precond_laplacian<T>(ctx, alpha, (const cplx<T>*)r, (cplx<T>*)z, nrhs, nullptr, part));
  } else {
    // this energy's mode table in the workspace (the context's cached tables
    // are left alone), checked for thresholds on the host
    ModeData* modes = (ModeData*)(ws + o_modes);
    int* flag = (int*)(ws + o_modes + align256((size_t)nxy * sizeof(ModeData)));
    const double* E_d = (const double*)upload_bytes(ctx, 60, &E, sizeof(double));
    HIPCHK(launch_modes(ctx, E_d, 1, modes));
    hipLaunchKernelGGL(k_mode_flags_or, dim3(1), dim3(256), 0, ctx->stream, modes, nxy, flag);
    HIPCHK(hipGetLastError());
    int* flag_h = (int*)((char*)ctx->arena_h + 61 * kRegion);
    HIPCHK(hipMemcpyAsync(flag_h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    if (flag_h[0] & MODE_THRESHOLD) {
      char buf[128];
      snprintf(buf, sizeof buf, "energy %.12g is at a lateral channel threshold", E);
      ctx->err = buf;
      throw Fail{IOBM_E_AT_THRESHOLD};
    }
    if (flag_h[0] & MODE_FAIL) {
      ctx->err = "mode setup failed";
      throw Fail{IOBM_E_DEVICE};
    }
    // every vector uses mode table entry 0: an array of nrhs zeros in region 59
    int* e_h = (int*)((char*)ctx->arena_h + 59 * kRegion);
    if (ctx->region_pending[59]) stream_sync(ctx);
    memset(e_h, 0, (size_t)nrhs * sizeof(int));
    int* e_d = (int*)((char*)ctx->arena_d + 59 * kRegion);
    HIPCHK(hipMemcpyAsync(e_d, e_h, (size_t)nrhs * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    ctx->region_pending[59] = 1;
    HIPCHK(launch_precond_fft<T>(ctx, (const cplx<T>*)r, (cplx<T>*)z, (cplx<T>*)(ws + o_pf), nrhs, e_d, modes,
                                 nullptr, part));
  }
  if (rz) {
    hipLaunchKernelGGL(k_sum_partials, dim3((nrhs + 63) / 64), dim3(64), 0, ctx->stream, part, nrhs, slots, rz_d);
    HIPCHK(hipGetLastError());
    double* rz_h = (double*)((char*)ctx->arena_h + 62 * kRegion);
    HIPCHK(hipMemcpyAsync(rz_h, rz_d, (size_t)nrhs * 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    stream_sync(ctx);
    memcpy(rz, rz_h, (size_t)nrhs * 2 * sizeof(double));
  }
}

}  // namespace

extern "C" iobm_status iobm_precondition_noalloc(iobm_ctx ctx, int32_t precond, double alpha, double E,
                                                 int32_t nrhs, const void* r, void* z, int32_t precision,
                                                 double* rz) {
  if (!ctx) return IOBM_E_INVALID_ARG;
  if (nrhs < 0 || (nrhs > 0 && (!r || !z)) || !isfinite(E) || !(alpha > 0) ||
      (precision != IOBM_C128 && precision != IOBM_C64_REFINED) || precond < 0 || precond > 2)
    return fail(ctx, IOBM_E_INVALID_ARG, "bad arguments");
  if (r == z) return fail(ctx, IOBM_E_INVALID_ARG, "r and z must not overlap");
  if (!ctx->static_ws) return fail(ctx, IOBM_E_BAD_STATE, "no static workspace on this device");
  if (nrhs == 0) return IOBM_OK;
  const int prof = ctx->prof_mask;  // the timing hook records events: off for this call
  ctx->prof_mask = 0;
  iobm_status st = IOBM_OK;
  try {
    if (precision == IOBM_C128) precondition_static<double>(ctx, precond, alpha, E, nrhs, r, z, rz);
    else precondition_static<float>(ctx, precond, alpha, E, nrhs, r, z, rz);
  } catch (Fail& f) {
    st = f.s;
  }
  ctx->prof_mask = prof;
  return st;
}
