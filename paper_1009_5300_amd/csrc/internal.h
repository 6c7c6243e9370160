// Internal declarations of libiobm (not part of the ABI).
#pragma once

#include <algorithm>
#include <string>
#include <vector>

#include "common.h"
#include "iobm.h"

// Per (energy, lateral mode) electrode data, FP64.  Produced on the device
// by the mode-setup kernel from the lead dispersion (Eqs. (12)-(15)
// generalised to FD order 2*nf).  Plane index conventions: right-electrode
// blocks act on planes nz-nf+i (i = 0..nf-1); the left electrode is the
// mirror image.
struct ModeData {
  zd sig[9];   // Sigma_R block, row-major nf x nf (Sigma_L = reversed planes)
  zd q[3];     // monic polynomial of the nf outgoing Bloch roots: x^nf + sum_k q_k x^k
  zd fb[3];    // flat-wire Green's function filter numerator, d = 0..nf-1 (causal part)
  zd fbb[3];   // same for the anti-causal part (distances >= 1)
  zd lr[3];    // readout row: transmitted amplitude at plane nz-nf from planes nz-nf+m
  zd ll[3];    // readout row: reflected amplitude at plane 0 from planes m
  zd btil[3];  // right-hand side profile on planes 0..nf-1 (unit incident amplitude)
  zd xp;       // propagating outgoing root exp(i k_z h_z) (0 if closed)
  zd kin;      // reflected-basis projection of the incident wave itself
  double eps;  // lateral kinetic energy
  double v;    // group velocity of the propagating state (0 if closed)
  int flags;   // bit 0 open, bit 1 at threshold, bit 2 root failure
  int pad_;
};

enum { MODE_OPEN = 1, MODE_THRESHOLD = 2, MODE_FAIL = 4 };

struct ModeArgs {
  int nx, ny, nf, nE;
  double hx, hy, hz;
  double c[4];
  // lateral Bloch vector of the entry as phases per lattice step,
  // kappa_x h_x and kappa_y h_y (Eqs. (12)-(13) at G + kappa); 0 by default
  double tx = 0, ty = 0;
};
__host__ __device__ void compute_mode(const ModeArgs& A, double E, int m, ModeData* out);

struct KBData {
  int ncen = 0, rank = 0, nproj = 0;
  int nu = 0;             // voxels in the union of supports
  int* uvox = nullptr;    // [nu] flat voxel ids (device)
  double* Bd = nullptr;   // [nu][nproj_pad] projector values, zero where off-support
  float* Bf = nullptr;
  double* Btd = nullptr;  // [nproj][nu] the same values transposed (back-projection)
  float* Btf = nullptr;
  int* ctile = nullptr;   // [chunks of 64 union voxels] bit t: projector tile t has a nonzero value there
  int* prange = nullptr;  // [blocks of 256 union voxels][2] projectors [lo, hi) with nonzero values there
  double* hD = nullptr;   // [nproj][nproj] block-diagonal h^3 D (device)
  double* diag_d = nullptr;  // [npts] diagonal of B h^3 D B^T (device; Jacobi preconditioner)
  int nproj_pad = 0;      // nproj rounded up to the MFMA tile (multiple of 16)
};

// Device workspace pointers that grow with the number of right-hand sides.
struct Work {
  size_t bytes = 0;
  void* base = nullptr;
};

struct iobm_ctx_s {
  GridDev g;
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cu = 256;  // compute units of the device
  double c[4];     // central FD weights chat_0..chat_nf (h = 1)
  FFTPlan2D plan;
  zd* twx_d = nullptr;  // exp(-2 pi i k / nx), k < nx
  zd* twy_d = nullptr;
  zf* twx_f = nullptr;
  zf* twy_f = nullptr;
  // blocks per rhs of the z filter's paired layout (zpair_mode; 0: off)
  int zpair_nmb = 0;
  double* V_d = nullptr;
  float* V_f = nullptr;
  bool have_V = false;
  KBData kb;
  // cached mode tables for the most recent energy list
  std::vector<double> modeE;
  std::vector<double> modeK;  // per entry (kappa_x h_x, kappa_y h_y); empty when every kappa is 0
  ModeData* modes_d = nullptr;
  std::vector<ModeData> modes_h;
  size_t modes_cap = 0;
  // Sigma_R blocks of the same energies, [energy][nf * nf][mode], in both
  // precisions (coalesced reads for the electrode kernels)
  zd* sig_d = nullptr;
  zf* sig_f = nullptr;
  size_t sig_cap = 0;
  int* mode_flags_d = nullptr;       // ModeData::flags of the same table, [energy][mode]
  zd* sdiag_d = nullptr;             // [energy][nf] real-space diagonal of Sigma_R per face plane
  std::vector<int> mode_flags_h;     // host copy (the solve path needs only these)
  bool modes_h_valid = false;        // modes_h is copied from the device on demand
  void* arena_d = nullptr;  // small index arrays (device) and their pinned host mirror
  void* arena_h = nullptr;
  void* rb_h = nullptr;     // pinned host buffer for the solver's per-rhs read-backs
  size_t rb_cap = 0;
  unsigned char region_pending[64] = {0};
  // launch shapes per iteration precision (index prec_index<T>(): 0
  // complex128, 1 complex64); fields 0 = the default rule.  `tuned` is set
  // once the autotuner has run or a shape was pinned (the autotuner then
  // leaves the shape alone).
  iobm_launch_shape shape[2] = {};
  bool tuned[2] = {false, false};
  bool pinned[2] = {false, false};
  // kernel timing hook
  int prof_mask = 0;
  std::vector<hipEvent_t> prof_ev;  // start/stop pairs
  std::vector<int> prof_cls;        // class of each pair
  std::vector<double> prof_bytes;   // pass bytes of each pair
  size_t prof_used = 0;             // pairs recorded
  // pooled device scratch
  std::vector<std::pair<void*, size_t>> pool;
  // the library's own stream and events for graph-captured iterations
  // (created on first use; the caller's stream may be the null stream,
  // which cannot be captured)
  hipStream_t cap_stream = nullptr;
  hipEvent_t cap_ev[2] = {nullptr, nullptr};
  // device address of this device's copy of the library's static workspace
  // (iobm_precondition_noalloc), looked up once per device
  void* static_ws = nullptr;
  std::string err;
};

// Pair j of the z filter's paired layout, member h (0: the mode k, 1: its
// partner -k), as a mode index of the natural FFT order m = iy nx + ix, or
// nxy past the last pair.  The pairs are, in order: row 0 with 1 <= ix <=
// (nx-1)/2; rows 1 .. (ny-1)/2, every ix; row ny/2 (even ny) with 1 <= ix <=
// (nx-1)/2; then the self-paired modes (k = -k: ix in {0, nx/2}, iy in
// {0, ny/2}), two to a pair, flagged in self.  Every other mode is the
// partner of one of these.
__host__ __device__ inline int zpair_mode(int j, int h, int ny, int nx, bool& self) {
  const int nxy = nx * ny, r0 = (nx - 1) / 2, nb = ((ny - 1) / 2) * nx;
  const int nc = (ny % 2 == 0) ? r0 : 0;
  const int npair = r0 + nb + nc;
  self = false;
  if (j < npair) {
    int ix, iy;
    if (j < r0) { ix = j + 1; iy = 0; }
    else if (j < r0 + nb) { iy = 1 + (j - r0) / nx; ix = (j - r0) % nx; }
    else { ix = j - r0 - nb + 1; iy = ny / 2; }
    if (h) { ix = (nx - ix) % nx; iy = (ny - iy) % ny; }
    return iy * nx + ix;
  }
  // self-paired modes: (0,0), (nx/2,0) for even nx, (0,ny/2) for even ny, (nx/2,ny/2) for both
  const int sx = (nx % 2 == 0) ? 2 : 1, sy = (ny % 2 == 0) ? 2 : 1;
  const int si = 2 * (j - npair) + h;
  if (si >= sx * sy) return nxy;
  self = true;
  return (si / sx) * (ny / 2) * nx + (si % sx) * (nx / 2);
}

template <typename T> constexpr int prec_index() { return sizeof(T) == sizeof(float) ? 1 : 0; }

// FD stencil of the operator A_st = E - V - T (Eq. (1) with the central
// weights chat_n / h_mu^2): e0 = the diagonal kinetic term, w*[n] the
// coupling to the neighbours at distance n per direction; the volume
// kernels run over chunks of zchunk planes per right-hand side.
struct StencilArgs {
  int nx, ny, nz, nf, nxy;
  int zchunk, nchunks;
  double e0;
  double wx[4], wy[4], wz[4];
};
StencilArgs stencil_args(iobm_ctx c, int zchunk);

// Bond phases of the lateral couplings in the gauge u = exp(-i kappa.r) psi
// of a lateral Bloch vector kappa: x[n] = exp(i n kappa_x h_x),
// y[n] = exp(i n kappa_y h_y), n = 1..3 (index 0 unused); the rhs at -kappa
// take the conjugates.
struct BlochPhase {
  zd x[4], y[4];
};

// ---- kernel timing hook (api.hip) -------------------------------------------
// prof_start records a start event for one launch of class cls and returns
// its record (or -1 when the class is not timed); prof_stop records the end
// and the launch's algorithmic bytes (every vector it must read or write,
// once).  Records may nest.
int prof_start(iobm_ctx c, int cls);
void prof_stop(iobm_ctx c, int rec, double alg_bytes);

// ---- launchers (ops.hip / modes.hip / kb.hip) -------------------------------
struct RhsMap {        // device arrays describing a batch of right-hand sides
  const int* energy;   // [nrhs] index into the mode table
  const double* E;     // [nrhs] energy
};

// kap_d: per entry (kappa_x h_x, kappa_y h_y), or nullptr for kappa = 0
hipError_t launch_modes(iobm_ctx c, const double* E_d, int nE, ModeData* out, const double* kap_d = nullptr);
hipError_t launch_sigma_tables(iobm_ctx c, int nE, const ModeData* modes, zd* sig_d, zf* sig_f, int* flags);

// Per-rhs FP64 partial sums of a bilinear form u^T v (re, im) and of |u|^2
// (n2), one per block, combined in a fixed order.
struct Partial {
  double re, im, n2, pad;
};

// Slots of the per-rhs partials of mu = p^T A p written by the fused
// operator: stencil chunks [0, PQ_STENCIL_MAX), the two electrode faces at
// PQ_BOUNDARY and PQ_BOUNDARY + 1, the nonlocal term at PQ_KB.  Unused
// slots hold zeros (the buffer is cleared once per solve).
enum { PQ_STENCIL_MAX = 64, PQ_BOUNDARY = 64, PQ_KB = 66, PQ_SLOTS = 68 };

// Fused COCG direction update for launch_apply: the operand is
// pnew = z + beta p_old (beta per rhs; p_old is not read where beta = 0),
// written to pnew, and the partials of pnew^T (A pnew) go to part.  With
// alpha, d and dlive set, the previous step's update d += alpha p_old is
// applied on the way (per rhs; none where alpha = 0; d is not read where
// dlive = 0, the first step after a refinement).  For the byte count of the
// timing hook: nfresh of the rhs restart here (beta = alpha = 0), nkept
// continue their direction right after a replacement (alpha = 0, beta != 0),
// nfirstd make their first d update.
template <typename T>
struct ApplyFuse {
  const cplx<T>* z;
  const cplx<T>* pold;
  const zd* beta;
  cplx<T>* pnew;
  Partial* part;  // [rhs][PQ_SLOTS]
  const zd* alpha = nullptr;
  cplx<T>* d = nullptr;
  const int* dlive = nullptr;
  int nfresh = 0;
  int nfirstd = 0;
  int nkept = 0;
};

template <typename T>
hipError_t launch_apply(iobm_ctx c, const cplx<T>* x, cplx<T>* y, int nrhs, const double* E_rhs,
                        const int* e_rhs, const ModeData* modes, const int* active,
                        const ApplyFuse<T>* fuse = nullptr);
// The preconditioners optionally write the per-rhs partials of r^T z to
// dpart (precond_slots(c, pc) per rhs).
template <typename T>
hipError_t launch_precond_laplacian(iobm_ctx c, double alpha, const cplx<T>* r, cplx<T>* z,
                                    int nrhs, const int* active, Partial* dpart = nullptr);
template <typename T>
hipError_t launch_precond_jacobi(iobm_ctx c, const cplx<T>* r, cplx<T>* z, int nrhs, const int* e_rhs,
                                 const double* E_rhs, const int* active, Partial* dpart = nullptr);
hipError_t launch_sigma_diag(iobm_ctx c, int nE);  // sdiag_d from sig_d for the current table
// y = A_st p_new with lateral bond phases (the gauge of a lateral Bloch
// vector; sgn[rhs] < 0 selects -kappa), with the pair iteration's direction
// update fused: p_new = z + beta p_old written to pnew, and the pending
// correction d += alpha p_old (beta, alpha per pair; both zero after a
// restart, when p_old and d are not read; d is the FP64 solution itself in
// complex128)
template <typename T>
struct BlochFuse {
  const cplx<T>* z;
  const cplx<T>* pold;
  cplx<T>* pnew;
  cplx<T>* d;
  const zd* beta;
  const zd* alpha;
  int nfresh;  // slots restarted since their last step (byte count of the timing hook only)
};
template <typename T>
hipError_t launch_bloch_stencil_fused(iobm_ctx c, const BlochPhase& ph, const BlochFuse<T>& F, cplx<T>* y, int nrhs,
                                      const double* E_rhs, const int* sgn, const int* active);
// The pair restart's true residual at a lateral Bloch vector: r = b - A x
// from the FP64 solution with the phased stencil and the electrode term,
// stored in the iteration precision TR (b supported on the 2 nf face planes;
// rface holds the faces in FP64 on the way); |r|^2 partials per rhs in the
// operator layout (stencil chunk slots and the two faces of PQ_SLOTS)
template <typename TR>
hipError_t launch_bloch_refresh(iobm_ctx c, const BlochPhase& ph, const zd* x, const zd* b, zd* rface, cplx<TR>* r,
                                int nrhs, const double* E_rhs, const int* e_rhs, const int* sgn, const int* active,
                                Partial* part);
// y -= Sigma x on the 2 nf face planes, for the listed rhs
template <typename T>
hipError_t launch_face_sigma(iobm_ctx c, const cplx<T>* x, cplx<T>* y, int nrhs, const int* e_rhs, const int* active);
hipError_t launch_rhs(iobm_ctx c, int nrhs, const int* e_rhs, const int* mode_rhs, const int* kind_rhs, int side,
                      const ModeData* modes, zd* b, bool faces_only);
hipError_t launch_readout(iobm_ctx c, int nrhs, int side, const zd* x, const ModeData* modes, const int* e_rhs,
                          zd* amp_near, zd* amp_far);
int dot_blocks(iobm_ctx c);
// The COCG residual update fused into the preconditioner's forward transform
// (square planes of the register FFT only, see fft_reg_available): the
// residual, kept in lateral mode space in the preconditioner's scratch
// (R = FFT(r)), is updated from q, R -= alpha FFT(q).  The per-plane partials
// of |r|^2 go to n2part[rhs][nz].
template <typename T>
struct FftUpd {
  const cplx<T>* q = nullptr;
  const zd* alpha = nullptr;
  Partial* n2part = nullptr;
};
template <typename T>
bool fft_reg_available(iobm_ctx c);
template <typename T>
hipError_t launch_precond_fft(iobm_ctx c, const cplx<T>* r, cplx<T>* z, cplx<T>* scratch,
                              int nrhs, const int* e_rhs, const ModeData* modes,
                              const int* active, Partial* dpart = nullptr, const FftUpd<T>* upd = nullptr);
int precond_slots(iobm_ctx c, int precond);
template <typename T>
hipError_t launch_kb_apply(iobm_ctx c, const cplx<T>* x, cplx<T>* y, int nrhs, Partial* pq_part,
                           const int* active);
// Times the admissible stencil shapes (on the fused operator when `fuse` is
// given; its buffers are overwritten) and z-filter chunk lengths once per
// context and precision, unless a shape is pinned.
template <typename T>
void autotune(iobm_ctx c, const cplx<T>* x, cplx<T>* y, cplx<T>* scratch, int nrhs, const double* E_rhs,
              const int* e_rhs, const ModeData* modes, const int* active, const ApplyFuse<T>* fuse = nullptr,
              Partial* rz_part = nullptr);
size_t kb_proj_bytes(iobm_ctx c, int nrhs);
// Launch-shape rules (ops.hip): whether a pinned shape is admissible for
// this grid, and the shape in effect (pinned, tuned or the default rule).
bool launch_shape_valid(iobm_ctx c, int prec, const iobm_launch_shape& s, std::string& why);
iobm_launch_shape launch_shape_in_effect(iobm_ctx c, int prec);
double* kb_scratch(iobm_ctx c, size_t bytes);  // context-owned scratch for the projector sums
