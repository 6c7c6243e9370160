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
// The projection runs on the matrix cores: each wavefront owns a 16-voxel
// slab and accumulates the 16 x 16 block Bmat^T X for 16 projector columns
// and 8 complex right-hand sides (16 real columns) with
// v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 over 4-voxel steps.
#include "internal.h"

namespace {

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

// One wavefront (64 lanes) per block.  Block (slot group g, projector tile pt,
// K split ks).  16 real columns = 8 complex rhs (re, im interleaved).
// MFMA 16x16x4 operand layout (wave64): lane l holds A[row = l % 16][k = l / 16]
// and B[k = l / 16][col = l % 16]; accumulator rows per Mfma<T>::row.
template <typename T>
__global__ void __launch_bounds__(64) k_kb_project(KBData kb, long long vol, int nact, int ksplit,
                                                   const cplx<T>* __restrict__ x,
                                                   double* __restrict__ part,
                                                   const int* __restrict__ active) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int ngroups = (nact + 7) / 8;
  const int g = blockIdx.x % ngroups;
  const int pt = (blockIdx.x / ngroups) % (kb.nproj_pad / 16);
  const int ks = blockIdx.x / (ngroups * (kb.nproj_pad / 16));
  const int lane = threadIdx.x;
  const int col = lane & 15;         // real column: rhs slot g*8 + col/2, component col&1
  const int kk = lane >> 4;          // k within the 4-step
  const int slot = g * 8 + (col >> 1);
  const bool has = slot < nact;
  const int rhs = has ? (active ? active[slot] : slot) : 0;
  const T* B = bmat<T>(kb);
  const int per = (kb.nu + ksplit - 1) / ksplit;
  const int u0 = ks * per, u1 = min(kb.nu, u0 + per);
  acc_t acc = {0, 0, 0, 0};
  for (int u = u0; u < u1; u += 4) {
    const int uu = u + kk;
    T a = 0, b = 0;
    if (uu < u1) {
      a = B[(long long)uu * kb.nproj_pad + pt * 16 + col];  // A^T: row = projector, k = voxel
      if (has) {
        cplx<T> xv = x[rhs * vol + kb.uvox[uu]];
        b = (col & 1) ? xv.im : xv.re;
      }
    }
    acc = Mfma<T>::mma(a, b, acc);
  }
  // acc[i] = C[proj = pt*16 + row(lane, i)][real column = lane % 16]
  if (has) {
    for (int i = 0; i < 4; ++i) {
      const int p = pt * 16 + Mfma<T>::row(lane, i);
      part[(((long long)ks * nact + slot) * kb.nproj_pad + p) * 2 + (col & 1)] = (double)acc[i];
    }
  }
}

// Sum the K-split partials in fixed order, then W = (h^3 D) C, FP64.  With
// pq set, also the nonlocal part of x^T (A x), which is -C^T W, to
// pq[rhs][PQ_KB].
__global__ void k_kb_scale(KBData kb, int nact, int ksplit, const double* __restrict__ part,
                           double* __restrict__ W, Partial* __restrict__ pq,
                           const int* __restrict__ active) {
  const int slot = blockIdx.x;
  const int p = threadIdx.x;
  __shared__ double C[2 * 128];
  __shared__ double Wsh[2 * 128];
  if (p < kb.nproj_pad) {
    double re = 0, im = 0;
    for (int s = 0; s < ksplit; ++s) {
      re += part[(((long long)s * nact + slot) * kb.nproj_pad + p) * 2 + 0];
      im += part[(((long long)s * nact + slot) * kb.nproj_pad + p) * 2 + 1];
    }
    C[2 * p] = re;
    C[2 * p + 1] = im;
  }
  __syncthreads();
  if (p < kb.nproj_pad) {
    double re = 0, im = 0;
    if (p < kb.nproj) {
      for (int q = 0; q < kb.nproj; ++q) {
        double d = kb.hD[p * kb.nproj + q];
        re += d * C[2 * q];
        im += d * C[2 * q + 1];
      }
    }
    W[((long long)slot * kb.nproj_pad + p) * 2] = re;
    W[((long long)slot * kb.nproj_pad + p) * 2 + 1] = im;
    Wsh[2 * p] = re;
    Wsh[2 * p + 1] = im;
  }
  if (!pq) return;
  __syncthreads();
  if (threadIdx.x == 0) {
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

// y[rhs][vox(u)] -= sum_p Bmat[u][p] W[rhs][p]; union voxels are distinct, so
// no two threads touch the same element.
template <typename T>
__global__ void k_kb_back(KBData kb, long long vol, int nact, const double* __restrict__ W,
                          cplx<T>* __restrict__ y, const int* __restrict__ active) {
  const int slot = blockIdx.y;
  const int rhs = active ? active[slot] : slot;
  extern __shared__ double Ws[];
  for (int i = threadIdx.x; i < 2 * kb.nproj_pad; i += blockDim.x)
    Ws[i] = W[(long long)slot * kb.nproj_pad * 2 + i];
  __syncthreads();
  const T* B = bmat<T>(kb);
  for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < kb.nu; u += gridDim.x * blockDim.x) {
    T re = 0, im = 0;
    for (int p = 0; p < kb.nproj; ++p) {
      T b = B[(long long)u * kb.nproj_pad + p];
      re += b * (T)Ws[2 * p];
      im += b * (T)Ws[2 * p + 1];
    }
    cplx<T>* yp = y + rhs * vol + kb.uvox[u];
    cplx<T> v = *yp;
    *yp = mk<T>(v.re - re, v.im - im);
  }
}

}  // namespace

static int kb_ksplit(const KBData& kb) {
  int s = kb.nu / 512;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
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
  const KBData& kb = c->kb;
  const int ks = kb_ksplit(kb);
  size_t part_elems = (size_t)ks * nrhs * kb.nproj_pad * 2;
  double* part = kb_scratch(c, kb_proj_bytes(c, nrhs));
  if (!part) return hipErrorOutOfMemory;
  double* W = part + part_elems;
  const int ngroups = (nrhs + 7) / 8;
  dim3 g1(ngroups * (kb.nproj_pad / 16) * ks);
  const int rec = prof_start(c, sizeof(T) == 4 ? IOBM_K_NONLOCAL : IOBM_K_NONLOCAL_C128);
  hipLaunchKernelGGL(k_kb_project<T>, g1, dim3(64), 0, c->stream, kb, c->g.npts, nrhs, ks, x, part, active);
  // algorithmic flops of the real GEMM: M = projectors, N = 2 nrhs, K = support
  prof_stop(c, rec, 2.0 * kb.nproj * (2.0 * nrhs) * kb.nu);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_kb_scale, dim3(nrhs), dim3(128), 0, c->stream, kb, nrhs, ks, part, W, pq_part, active);
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  int bx = (kb.nu + 255) / 256;
  if (bx > 64) bx = 64;
  hipLaunchKernelGGL(k_kb_back<T>, dim3(bx, nrhs), dim3(256), 2 * kb.nproj_pad * sizeof(double), c->stream,
                     kb, c->g.npts, nrhs, W, y, active);
  return hipGetLastError();
}

template hipError_t launch_kb_apply<double>(iobm_ctx, const zd*, zd*, int, Partial*, const int*);
template hipError_t launch_kb_apply<float>(iobm_ctx, const zf*, zf*, int, Partial*, const int*);
