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
};
__host__ __device__ void compute_mode(const ModeArgs& A, double E, int m, ModeData* out);

struct KBData {
  int ncen = 0, rank = 0, nproj = 0;
  int nu = 0;             // voxels in the union of supports
  int* uvox = nullptr;    // [nu] flat voxel ids (device)
  double* Bd = nullptr;   // [nu][nproj_pad] projector values, zero where off-support
  float* Bf = nullptr;
  double* hD = nullptr;   // [nproj][nproj] block-diagonal h^3 D (device)
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
  double* V_d = nullptr;
  float* V_f = nullptr;
  bool have_V = false;
  KBData kb;
  // cached mode tables for the most recent energy list
  std::vector<double> modeE;
  ModeData* modes_d = nullptr;
  std::vector<ModeData> modes_h;
  size_t modes_cap = 0;
  // Sigma_R blocks of the same energies, [energy][nf * nf][mode], in both
  // precisions (coalesced reads for the electrode kernels)
  zd* sig_d = nullptr;
  zf* sig_f = nullptr;
  size_t sig_cap = 0;
  int* mode_flags_d = nullptr;       // ModeData::flags of the same table, [energy][mode]
  std::vector<int> mode_flags_h;     // host copy (the solve path needs only these)
  bool modes_h_valid = false;        // modes_h is copied from the device on demand
  void* arena_d = nullptr;  // small index arrays (device) and their pinned host mirror
  void* arena_h = nullptr;
  void* rb_h = nullptr;     // pinned host buffer for the solver's per-rhs read-backs
  size_t rb_cap = 0;
  unsigned char region_pending[64] = {0};
  // tuned launch shapes (0 = default rule)
  int tune_zf_c64 = 0, tune_zf_c128 = 0;
  int tune_fft_generic = 0;  // 1: always use the LDS Stockham plane FFT
  int tune_stencil_simple = 0;  // 1: cache-based stencil instead of the 2.5D one
  int tune_ppt_c64 = 0, tune_ppt_c128 = 0;  // 2.5D stencil points per thread (0 = default)
  int tune_zc_c64 = 0, tune_zc_c128 = 0;    // 2.5D stencil planes per block (0 = 32)
  bool tuned_c64 = false, tuned_c128 = false;
  // kernel timing hook
  int prof_mask = 0;
  std::vector<hipEvent_t> prof_ev;  // start/stop pairs
  std::vector<int> prof_cls;        // class of each pair
  std::vector<double> prof_bytes;   // pass bytes of each pair
  size_t prof_used = 0;             // pairs recorded
  // pooled device scratch
  std::vector<std::pair<void*, size_t>> pool;
  std::string err;
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

hipError_t launch_modes(iobm_ctx c, const double* E_d, int nE, ModeData* out);
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
// timing hook: nfresh of the rhs restart here (beta = alpha = 0), nfirstd
// make their first d update.
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
// context and precision.
template <typename T>
void autotune(iobm_ctx c, const cplx<T>* x, cplx<T>* y, cplx<T>* scratch, int nrhs, const double* E_rhs,
              const int* e_rhs, const ModeData* modes, const int* active, const ApplyFuse<T>* fuse = nullptr);
size_t kb_proj_bytes(iobm_ctx c, int nrhs);
double* kb_scratch(iobm_ctx c, size_t bytes);  // context-owned scratch for the projector sums
