// Separable nonlocal term y -= sum_a B_a (h^3 D_a) B_a^T x across a batch of
// right-hand sides (the pseudopotential part of H_T; Sec. III and IV use
// norm-conserving pseudopotentials in separable form).
//
// The projectors of all centres are stored densely on the union of their
// supports: Bmat[u][p] (u < nu union voxels, p < nproj_pad, zero where
// voxel u is outside centre a's sphere), so both contractions are dense
// GEMMs across right-hand sides:
//   projection      C[rhs][p] = sum_u Bmat[u][p] x[rhs][vox(u)]     (K = nu)
//   back-projection y[rhs][vox(u)] -= sum_p Bmat[u][p] W[rhs][p],  W = (h^3 D) C
// The union voxels are sorted by voxel id, so a run of consecutive union
// voxels of one right-hand side is mostly contiguous in memory.
//
// Projection: a block of four wavefronts owns 32 right-hand sides (8 per
// wavefront, 16 real columns) and one split of the union voxels, taken in
// chunks of 64.  Per chunk every wavefront loads its 8 right-hand sides
// with coalesced loads (lane = voxel), transposes them through LDS into the
// MFMA operand layout, and the four share one LDS copy of the chunk's
// projector rows.  v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 then
// accumulate all projector tiles over 4-voxel steps while the next chunk's
// loads are in flight.  The splits' partial sums are combined in a fixed
// order in FP64.
//
// Back-projection: a block owns 256 union voxels and 16 right-hand sides;
// it reads the projector values from a transposed copy Bmat^T[p][u]
// (coalesced), reuses each for the 16 right-hand sides, and updates y.
//
// Both skip where the projectors vanish: a centre's sphere covers a few runs
// of union voxels, so a chunk or block sees few centres.  Per 64-voxel chunk
// a mask of the nonzero projector tiles, per 256-voxel block the range of
// nonzero projectors (both set with the projectors) bound the work; what is
// skipped is exactly zero.
#include "internal.h"

namespace {

constexpr int KB_CH = 64;               // union voxels per chunk
constexpr int KB_WAVES = 4;             // wavefronts per projection block
constexpr int KB_GROUP = 8 * KB_WAVES;  // right-hand sides per projection block
constexpr int KB_XS = 18;               // LDS row stride of the transposed x chunk (16 columns + 2)
constexpr int KB_BACK_RHS = 16;         // right-hand sides per back-projection block

// LDS row stride of the projector chunk: the four k-rows of one MFMA step
// start 16 elements apart modulo 64, so their 16-lane reads use distinct
// banks.
__host__ __device__ constexpr int kb_bstride(int pad) { return (pad % 32 == 16) ? pad : pad + 16; }

template <typename T> struct Mfma;
// Accumulator layout (wave64): lane l holds D[row][l % 16] for its 4 values
// v; fp32 packs 4 consecutive rows per lane (row = 4 (l/16) + v), fp64 strides
// them by 4 (row = l/16 + 4 v).
template <> struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename T> __device__ __forceinline__ const T* bmat(const KBData& kb);
template <> __device__ __forceinline__ const double* bmat<double>(const KBData& kb) { return kb.Bd; }
template <> __device__ __forceinline__ const float* bmat<float>(const KBData& kb) { return kb.Bf; }
template <typename T> __device__ __forceinline__ const T* btmat(const KBData& kb);
template <> __device__ __forceinline__ const double* btmat<double>(const KBData& kb) { return kb.Btd; }
template <> __device__ __forceinline__ const float* btmat<float>(const KBData& kb) { return kb.Btf; }

// Registers of one chunk on its way from HBM to LDS: x of the wavefront's 8
// right-hand sides at voxel (chunk start + lane), and this thread's share of
// the projector rows as 16-byte vectors.
template <typename T, int NT>
struct KBStage {
  static constexpr int VEC = 16 / sizeof(T);                  // elements per 16-byte vector
  static constexpr int NB = KB_CH * NT * 16 / VEC / (64 * KB_WAVES);  // vectors per thread
  cplx<T> xv[8];
  uint4 bv[NB];
};

// Block: (group g of 32 right-hand-side slots, voxel split ks).  MFMA
// 16x16x4 operand layout (wave64): lane l holds A[row = l % 16][k = l / 16]
// and B[k = l / 16][col = l % 16]; A = Bmat^T (row = projector, k = voxel),
// B = X (k = voxel, col = real column: slot 8 w + col / 2, component col & 1).
template <typename T, int NT>
__global__ void __launch_bounds__(64 * KB_WAVES) k_kb_project(KBData kb, long long vol, int nact, int per,
                                                             const cplx<T>* __restrict__ x,
                                                             double* __restrict__ part,
                                                             const int* __restrict__ active) {
  typedef typename Mfma<T>::acc_t acc_t;
  typedef KBStage<T, NT> Stage;
  constexpr int PAD = NT * 16;
  constexpr int BS = kb_bstride(PAD);
  constexpr int VPR = PAD / Stage::VEC;  // 16-byte vectors per projector row
  extern __shared__ __align__(16) char kb_lds[];
  T* Bs = (T*)kb_lds;                 // [KB_CH][BS]
  T* xs = Bs + KB_CH * BS;            // [KB_WAVES][KB_CH][KB_XS]
  const int ngroups = (nact + KB_GROUP - 1) / KB_GROUP;
  const int g = blockIdx.x % ngroups;
  const int ks = blockIdx.x / ngroups;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int col = lane & 15, kk = lane >> 4;
  T* xw = xs + w * KB_CH * KB_XS;
  const int slot0 = g * KB_GROUP + w * 8;
  long long xoff[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int slot = slot0 + r;
    xoff[r] = slot < nact ? (long long)(active ? active[slot] : slot) * vol : -1;
  }
  const uint4* B4 = (const uint4*)bmat<T>(kb);
  const int u0 = ks * per, u1 = min(kb.nu, u0 + per);

  Stage st;
  // voxel ids run one chunk ahead of the x loads that depend on them
  auto ids = [&](int uc) { return uc + lane < u1 ? kb.uvox[uc + lane] : 0; };
  int vnext = ids(u0);
  auto load = [&](int uc) {
    const int u = uc + lane;
    const int vox = vnext;
    vnext = ids(uc + KB_CH);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      st.xv[r] = mk<T>(0, 0);
      if (u < u1 && xoff[r] >= 0) st.xv[r] = x[xoff[r] + vox];
    }
#pragma unroll
    for (int i = 0; i < Stage::NB; ++i) {
      const int j = t + i * 64 * KB_WAVES;
      const int row = j / VPR;
      st.bv[i] = make_uint4(0, 0, 0, 0);
      if (uc + row < u1) st.bv[i] = B4[(long long)(uc + row) * VPR + j % VPR];
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      xw[lane * KB_XS + 2 * r] = st.xv[r].re;
      xw[lane * KB_XS + 2 * r + 1] = st.xv[r].im;
    }
#pragma unroll
    for (int i = 0; i < Stage::NB; ++i) {
      const int j = t + i * 64 * KB_WAVES;
      *(uint4*)(Bs + (j / VPR) * BS + (j % VPR) * Stage::VEC) = st.bv[i];
    }
  };

  acc_t acc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) acc[tt] = acc_t{0, 0, 0, 0};
  if (u0 < u1) load(u0);
  for (int uc = u0; uc < u1; uc += KB_CH) {
    __syncthreads();  // the previous chunk's LDS reads are done
    store();
    __syncthreads();
    if (uc + KB_CH < u1) load(uc + KB_CH);  // in flight during this chunk's MFMAs
    T b[KB_CH / 4];
#pragma unroll
    for (int s = 0; s < KB_CH / 4; ++s) b[s] = xw[(4 * s + kk) * KB_XS + col];
    const int mask = kb.ctile[uc / KB_CH];  // tiles that are zero on this chunk add nothing
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      if (!(mask >> tt & 1)) continue;
#pragma unroll
      for (int s = 0; s < KB_CH / 4; ++s)
        acc[tt] = Mfma<T>::mma(Bs[(4 * s + kk) * BS + tt * 16 + col], b[s], acc[tt]);
    }
  }
  // acc[tt][i] = C[proj = tt*16 + row(lane, i)][real column = lane % 16];
  // every split writes its partial sums, zeros where its range is empty
  const int slot = slot0 + (col >> 1);
  if (slot < nact) {
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = tt * 16 + Mfma<T>::row(lane, i);
        part[(((long long)ks * nact + slot) * PAD + p) * 2 + (col & 1)] = (double)acc[tt][i];
      }
  }
}

// Sum the voxel-split partials in fixed order (each thread a strided subset
// of the splits, then the subsets in order), then W = (h^3 D) C in FP64
// over the centre's own rank x rank block.  With pq set, also the nonlocal
// part of x^T (A x), which is -C^T W, to pq[rhs][PQ_KB].
__global__ void __launch_bounds__(256) k_kb_scale(KBData kb, int nact, int ksplit, const double* __restrict__ part,
                                                  double* __restrict__ W, Partial* __restrict__ pq,
                                                  const int* __restrict__ active) {
  const int slot = blockIdx.x;
  const int nv = 2 * kb.nproj_pad;  // values per right-hand side (re, im per projector)
  const int nsl = 256 / nv;         // >= 1: nproj_pad <= 128
  __shared__ double red[256];
  __shared__ double C[256];
  __shared__ double Wsh[256];
  const int t = threadIdx.x;
  const int i = t % nv, sl = t / nv;
  if (sl < nsl) {
    double acc = 0;
#pragma unroll 8
    for (int s = sl; s < ksplit; s += nsl) acc += part[((long long)s * nact + slot) * nv + i];
    red[sl * nv + i] = acc;
  }
  __syncthreads();
  if (t < nv) {
    double c = 0;
    for (int k = 0; k < nsl; ++k) c += red[k * nv + t];
    C[t] = c;
  }
  __syncthreads();
  if (t < nv) {
    const int p = t >> 1, comp = t & 1;
    double acc = 0;
    if (p < kb.nproj) {
      const int q0 = p / kb.rank * kb.rank;
      for (int q = q0; q < q0 + kb.rank; ++q) acc += kb.hD[p * kb.nproj + q] * C[2 * q + comp];
    }
    W[(long long)slot * nv + t] = acc;
    Wsh[t] = acc;
  }
  if (!pq) return;
  __syncthreads();
  if (t == 0) {
    double re = 0, im = 0;
    for (int q = 0; q < kb.nproj; ++q) {
      re -= C[2 * q] * Wsh[2 * q] - C[2 * q + 1] * Wsh[2 * q + 1];
      im -= C[2 * q] * Wsh[2 * q + 1] + C[2 * q + 1] * Wsh[2 * q];
    }
    Partial P;
    P.re = re; P.im = im; P.n2 = 0; P.pad = 0;
    pq[(long long)(active ? active[slot] : slot) * PQ_SLOTS + PQ_KB] = P;
  }
}

// y[rhs][vox(u)] -= sum_p Bmat[u][p] W[rhs][p] for 256 union voxels and 16
// right-hand-side slots per block; union voxels are distinct, so no two
// threads touch the same element.
template <typename T>
__global__ void __launch_bounds__(256) k_kb_back(KBData kb, long long vol, int nact, const double* __restrict__ W,
                                                 cplx<T>* __restrict__ y, const int* __restrict__ active) {
  const int nv = 2 * kb.nproj_pad;
  const int slot0 = blockIdx.y * KB_BACK_RHS;
  extern __shared__ __align__(16) char kb_lds[];
  cplx<T>* Ws = (cplx<T>*)kb_lds;  // [nproj_pad][KB_BACK_RHS]
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const bool on = u < kb.nu;
  // y of this voxel for every slot, in flight while W is staged and the
  // projector sums run
  long long yoff[KB_BACK_RHS];  // per slot, the same in every lane
  cplx<T> yv[KB_BACK_RHS];
  const int vox = on ? kb.uvox[u] : 0;
#pragma unroll
  for (int r = 0; r < KB_BACK_RHS; ++r) {
    const int slot = slot0 + r;
    yoff[r] = slot < nact ? (long long)(active ? active[slot] : slot) * vol : -1;
    yv[r] = (on && yoff[r] >= 0) ? y[yoff[r] + vox] : mk<T>(0, 0);
  }
  for (int i = threadIdx.x; i < KB_BACK_RHS * kb.nproj_pad; i += blockDim.x) {
    const int p = i / KB_BACK_RHS, r = i % KB_BACK_RHS;
    const int slot = slot0 + r;
    cplx<T> v = mk<T>(0, 0);
    if (slot < nact) v = mk<T>((T)W[(long long)slot * nv + 2 * p], (T)W[(long long)slot * nv + 2 * p + 1]);
    Ws[i] = v;
  }
  __syncthreads();
  if (!on) return;
  const T* Bt = btmat<T>(kb);
  T re[KB_BACK_RHS], im[KB_BACK_RHS];
#pragma unroll
  for (int r = 0; r < KB_BACK_RHS; ++r) re[r] = im[r] = 0;
  // only the projectors that are nonzero somewhere in this block, their
  // values loaded 8 at a time
  const int plo = kb.prange[2 * blockIdx.x], phi = kb.prange[2 * blockIdx.x + 1];
  for (int p0 = plo; p0 < phi; p0 += 8) {
    T b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = p0 + j < phi ? Bt[(long long)(p0 + j) * kb.nu + u] : T(0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (p0 + j >= phi) break;
#pragma unroll
      for (int r = 0; r < KB_BACK_RHS; ++r) {
        const cplx<T> wv = Ws[(p0 + j) * KB_BACK_RHS + r];
        re[r] += b[j] * wv.re;
        im[r] += b[j] * wv.im;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < KB_BACK_RHS; ++r)
    if (yoff[r] >= 0) y[yoff[r] + vox] = mk<T>(yv[r].re - re[r], yv[r].im - im[r]);
}

template <typename T, int NT>
hipError_t launch_project(const KBData& kb, hipStream_t s, long long vol, int nact, int ks, int per,
                          const cplx<T>* x, double* part, const int* active) {
  constexpr int BS = kb_bstride(NT * 16);
  const size_t lds = (size_t)(KB_CH * BS + KB_WAVES * KB_CH * KB_XS) * sizeof(T);
  const int ngroups = (nact + KB_GROUP - 1) / KB_GROUP;
  hipLaunchKernelGGL((k_kb_project<T, NT>), dim3(ngroups * ks), dim3(64 * KB_WAVES), lds, s, kb, vol, nact, per,
                     x, part, active);
  return hipGetLastError();
}

}  // namespace

// Voxel splits of the projection: about 192 union voxels each, at most 128.
static int kb_ksplit(const KBData& kb) {
  int s = (kb.nu + 191) / 192;
  if (s < 1) s = 1;
  if (s > 128) s = 128;
  return s;
}

size_t kb_proj_bytes(iobm_ctx c, int nrhs) {
  if (c->kb.ncen == 0) return 0;
  size_t part = (size_t)kb_ksplit(c->kb) * nrhs * c->kb.nproj_pad * 2 * sizeof(double);
  size_t W = (size_t)nrhs * c->kb.nproj_pad * 2 * sizeof(double);
  return part + W;
}

template <typename T>
hipError_t launch_kb_apply(iobm_ctx c, const cplx<T>* x, cplx<T>* y, int nrhs, Partial* pq_part,
                           const int* active) {
  if (nrhs <= 0) return hipSuccess;
  const KBData& kb = c->kb;
  const int ks = kb_ksplit(kb);
  // split length in whole chunks; trailing splits may be empty (zero partials)
  const int per = ((kb.nu + ks - 1) / ks + KB_CH - 1) / KB_CH * KB_CH;
  size_t part_elems = (size_t)ks * nrhs * kb.nproj_pad * 2;
  double* part = kb_scratch(c, kb_proj_bytes(c, nrhs));
  if (!part) return hipErrorOutOfMemory;
  double* W = part + part_elems;
  const int rec = prof_start(c, sizeof(T) == 4 ? IOBM_K_NONLOCAL : IOBM_K_NONLOCAL_C128);
  hipError_t err;
  switch (kb.nproj_pad / 16) {
    case 1: err = launch_project<T, 1>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    case 2: err = launch_project<T, 2>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    case 3: err = launch_project<T, 3>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    case 4: err = launch_project<T, 4>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    case 5: err = launch_project<T, 5>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    case 6: err = launch_project<T, 6>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    case 7: err = launch_project<T, 7>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    case 8: err = launch_project<T, 8>(kb, c->stream, c->g.npts, nrhs, ks, per, x, part, active); break;
    default: return hipErrorInvalidValue;
  }
  // algorithmic flops of the real GEMM: M = projectors, N = 2 nrhs, K = support
  prof_stop(c, rec, 2.0 * kb.nproj * (2.0 * nrhs) * kb.nu);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_kb_scale, dim3(nrhs), dim3(256), 0, c->stream, kb, nrhs, ks, part, W, pq_part, active);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  dim3 gb((kb.nu + 255) / 256, (nrhs + KB_BACK_RHS - 1) / KB_BACK_RHS);
  hipLaunchKernelGGL(k_kb_back<T>, gb, dim3(256), (size_t)KB_BACK_RHS * kb.nproj_pad * sizeof(cplx<T>), c->stream,
                     kb, c->g.npts, nrhs, W, y, active);
  return hipGetLastError();
}

template hipError_t launch_kb_apply<double>(iobm_ctx, const zd*, zd*, int, Partial*, const int*);
template hipError_t launch_kb_apply<float>(iobm_ctx, const zf*, zf*, int, Partial*, const int*);
