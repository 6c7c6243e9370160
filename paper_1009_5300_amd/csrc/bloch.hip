// Kernels of the solve at a lateral Bloch vector kappa != 0 (Eqs. (2),
// (12)-(13) and (16) at G + kappa), in complex128 or in complex64 with FP64
// residual replacement (the pair recurrences run on a correction d of the
// FP64 solution x; every inner product is summed in FP64).
//
// Gauge.  The solve runs on u = exp(-i kappa.r) psi (r the lateral lattice
// position in the cell).  In this gauge the lateral Fourier transform of
// Eq. (16) at G + kappa is the plain FFT of u, so the electrode term, the
// lateral-Fourier preconditioner, the right-hand side and the readout are the
// kappa = 0 kernels run on a mode table built at G + kappa.  The Bloch
// condition psi(r + L) = exp(i kappa L) psi(r) turns into a periodic u whose
// lateral couplings carry a bond phase: the neighbour at +n along x enters
// with exp(i n kappa_x h_x), the one at -n with its conjugate.  Only the
// stencil (the 2.5D kernel with the OpBlochFuse policy, which also forms
// the direction and the pending correction of the pair iteration, and with
// OpBlochRefresh for a restart's residual; ops.hip) and Eq. (17) (this file)
// change; the diagonal (and so the Jacobi preconditioner) does not.
//
// Transpose.  A(kappa)^T = A(-kappa): the operator is not complex symmetric
// for one kappa, so each state at +kappa is solved together with a partner
// at -kappa by the bilinear biconjugate-gradient recurrence (the partner is
// the shadow system, A(kappa)^T y = c).  Pairs occupy two consecutive slots
// (primary 2k at +kappa, shadow 2k+1 at -kappa); the two slots share the
// scalars alpha, beta and rho of their pair.
#include "internal.h"

namespace {

__device__ __forceinline__ int bl_rhs(const int* active, int slot) { return active ? active[slot] : slot; }

// Block sum (whole wavefronts); the result is in thread 0.
__device__ __forceinline__ void bl_reduce3(double& a, double& b, double& c) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
    c += __shfl_xor(c, off);
  }
  __shared__ double sh[3][16];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { sh[0][w] = a; sh[1][w] = b; sh[2][w] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double ra = 0, rb = 0, rc = 0;
    for (int i = 0; i < nw; ++i) { ra += sh[0][i]; rb += sh[1][i]; rc += sh[2][i]; }
    a = ra; b = rb; c = rc;
  }
}

// Eq. (17) in the gauge u: z = r + c1 (sum of the six face neighbours), the
// lateral ones with the bond phase of distance 1, z neighbours outside the
// region zero.
template <typename T>
__global__ void __launch_bounds__(256) k_bl_laplacian(StencilArgs S, BlochPhase ph, double c1d,
                                                      const cplx<T>* __restrict__ r, cplx<T>* __restrict__ z,
                                                      const int* __restrict__ sgn, const int* __restrict__ active) {
  const int slot = blockIdx.x / S.nchunks;
  const int chunk = blockIdx.x - slot * S.nchunks;
  const int rhs = bl_rhs(active, slot);
  const long long vol = (long long)S.nxy * S.nz;
  const cplx<T>* rr = r + rhs * vol;
  cplx<T>* zr = z + rhs * vol;
  const bool neg = sgn[rhs] < 0;
  const cplx<T> px = cvt<T>(neg ? conj(ph.x[1]) : ph.x[1]);
  const cplx<T> py = cvt<T>(neg ? conj(ph.y[1]) : ph.y[1]);
  const T c1 = (T)c1d;
  const int z0 = chunk * S.zchunk;
  const int z1 = min(S.nz, z0 + S.zchunk);
  for (int k = z0; k < z1; ++k) {
    const cplx<T>* rp = rr + (long long)k * S.nxy;
    for (int p = threadIdx.x; p < S.nxy; p += blockDim.x) {
      const int j = p / S.nx;
      const int i = p - j * S.nx;
      int ip = i + 1; if (ip >= S.nx) ip -= S.nx;
      int im = i - 1; if (im < 0) im += S.nx;
      int jp = j + 1; if (jp >= S.ny) jp -= S.ny;
      int jm = j - 1; if (jm < 0) jm += S.ny;
      cplx<T> s = px * rp[j * S.nx + ip];
      s = cfma(conj(px), rp[j * S.nx + im], s);
      s = cfma(py, rp[jp * S.nx + i], s);
      s = cfma(conj(py), rp[jm * S.nx + i], s);
      if (k + 1 < S.nz) s = s + rp[S.nxy + p];
      if (k > 0) s = s + rp[-S.nxy + p];
      zr[(long long)k * S.nxy + p] = rp[p] + c1 * s;
    }
  }
}

// Per pair, partials of the bilinear form u(shadow)^T v(primary) over one
// contiguous chunk of the volume (FP64): part[pair][blk], pair = primary / 2.
template <typename T>
__global__ void __launch_bounds__(256) k_bl_dot(const cplx<T>* __restrict__ u, const cplx<T>* __restrict__ v,
                                                long long vol, int nblk, const int* __restrict__ pairs,
                                                Partial* __restrict__ part) {
  const int k = blockIdx.x / nblk;
  const int blk = blockIdx.x - k * nblk;
  const int prim = pairs[k];
  const long long per = (vol + nblk - 1) / nblk;
  const long long i0 = blk * per, i1 = min(vol, i0 + per);
  const cplx<T>* us = u + (long long)(prim + 1) * vol;
  const cplx<T>* vp = v + (long long)prim * vol;
  double re = 0, im = 0, d = 0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const cplx<T> a = us[i], b = vp[i];
    re += (double)a.re * b.re - (double)a.im * b.im;
    im += (double)a.re * b.im + (double)a.im * b.re;
  }
  bl_reduce3(re, im, d);
  if (threadIdx.x == 0) {
    Partial P;
    P.re = re; P.im = im; P.n2 = 0; P.pad = 0;
    part[(long long)(prim >> 1) * nblk + blk] = P;
  }
}

enum { BL_ALPHA = 0, BL_BETA = 1, BL_RESTART = 2 };

// Pair scalars from the partials, summed in a fixed order (one thread per
// pair):
//   BL_ALPHA:   mu = p~^T A p, alpha = rho / mu;
//   BL_BETA:    rho' = r~^T z, beta = rho' / rho, rho = rho', |r|^2 of both slots;
//   BL_RESTART: rho = r~^T z of a fresh residual, alpha = beta = 0, |r|^2
//               (from the residual operator's partials, PQ_SLOTS per slot:
//               the stencil chunks, then the two faces).
// A vanishing or non-finite denominator sets flag[pair] (the host restarts
// the pair from its true residual) and zeroes the step.
__global__ void __launch_bounds__(64) k_bl_scalars(int mode, int npairs, const int* __restrict__ pairs,
                                                   const Partial* __restrict__ pd, const Partial* __restrict__ pn,
                                                   int nblk, zd* __restrict__ rho, zd* __restrict__ alpha,
                                                   zd* __restrict__ beta, double* __restrict__ rn2,
                                                   int* __restrict__ flag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npairs) return;
  const int prim = pairs[k], pr = prim >> 1;
  zd s = mk(0.0, 0.0);
  for (int b = 0; b < nblk; ++b) s = s + mk(pd[(long long)pr * nblk + b].re, pd[(long long)pr * nblk + b].im);
  const bool finite = isfinite(s.re) && isfinite(s.im);
  if (mode == BL_ALPHA) {
    const double d = s.re * s.re + s.im * s.im;
    if (!finite || d == 0.0) {
      flag[pr] = 1;
      alpha[pr] = mk(0.0, 0.0);
    } else {
      const zd r = rho[pr];
      alpha[pr] = mk((r.re * s.re + r.im * s.im) / d, (r.im * s.re - r.re * s.im) / d);
    }
    return;
  }
  for (int sl = 0; sl < 2; ++sl) {
    double n = 0;
    if (mode == BL_RESTART) {
      const Partial* q = pn + (long long)(prim + sl) * PQ_SLOTS;
      for (int c = 0; c < PQ_STENCIL_MAX; ++c) n += q[c].n2;
      n += q[PQ_BOUNDARY].n2 + q[PQ_BOUNDARY + 1].n2;
    } else {
      for (int b = 0; b < nblk; ++b) n += pn[(long long)(prim + sl) * nblk + b].n2;
    }
    rn2[prim + sl] = n;
  }
  if (mode == BL_RESTART) {
    rho[pr] = s;
    alpha[pr] = mk(0.0, 0.0);
    beta[pr] = mk(0.0, 0.0);
    flag[pr] = (!finite || (s.re == 0.0 && s.im == 0.0)) ? 1 : 0;
    return;
  }
  const zd r = rho[pr];
  const double d = r.re * r.re + r.im * r.im;
  if (!finite || d == 0.0) {
    flag[pr] = 1;
    beta[pr] = mk(0.0, 0.0);
  } else {
    beta[pr] = mk((s.re * r.re + s.im * r.im) / d, (s.im * r.re - s.re * r.im) / d);
    rho[pr] = s;
  }
}

// r -= alpha q (alpha of the slot's pair), with the partials of |r|^2 in
// pn[slot][blk]; the matching d += alpha p is left to the next fused
// operator pass (or the settle of a restart).
template <typename T>
__global__ void __launch_bounds__(256) k_bl_update(cplx<T>* __restrict__ r, const cplx<T>* __restrict__ q,
                                                   const zd* __restrict__ alpha, long long vol, int nblk,
                                                   const int* __restrict__ active, Partial* __restrict__ pn) {
  const int slot = blockIdx.x / nblk;
  const int blk = blockIdx.x - slot * nblk;
  const int rhs = bl_rhs(active, slot);
  const cplx<T> a = cvt<T>(alpha[rhs >> 1]);
  const long long per = (vol + nblk - 1) / nblk;
  const long long i0 = blk * per, i1 = min(vol, i0 + per);
  const long long o = (long long)rhs * vol;
  double n2 = 0, d0 = 0, d1 = 0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const cplx<T> v = r[o + i] - a * q[o + i];
    r[o + i] = v;
    n2 += (double)v.re * v.re + (double)v.im * v.im;
  }
  bl_reduce3(n2, d0, d1);
  if (threadIdx.x == 0) {
    Partial P;
    P.re = 0; P.im = 0; P.n2 = n2; P.pad = 0;
    pn[(long long)rhs * nblk + blk] = P;
  }
}

// The pending correction folded into the FP64 solution: x += d + alpha p,
// d = 0 (complex64; alpha of the slot's pair), or x += alpha p (complex128,
// d == nullptr: the recurrence updates x itself).  p is not read where
// alpha = 0 (it may hold anything after a restart).
template <typename T>
__global__ void __launch_bounds__(256) k_bl_settle(zd* __restrict__ x, cplx<T>* __restrict__ d,
                                                   const cplx<T>* __restrict__ p, const zd* __restrict__ alpha,
                                                   long long vol, int nblk, const int* __restrict__ active) {
  const int slot = blockIdx.x / nblk;
  const int blk = blockIdx.x - slot * nblk;
  const int rhs = bl_rhs(active, slot);
  const zd a = alpha[rhs >> 1];
  const bool pend = a.re != 0.0 || a.im != 0.0;
  if (!d && !pend) return;
  const long long per = (vol + nblk - 1) / nblk;
  const long long i0 = blk * per, i1 = min(vol, i0 + per);
  const long long o = (long long)rhs * vol;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    zd v = x[o + i];
    if (d) {
      v = v + cvt<double>(d[o + i]);
      d[o + i] = mk<T>(0, 0);
    }
    if (pend) v = cfma(a, cvt<double>(p[o + i]), v);
    x[o + i] = v;
  }
}

}  // namespace

// =================================================================== host ===
template <typename T>
hipError_t launch_bloch_apply_fused(iobm_ctx c, const BlochPhase& ph, const BlochFuse<T>& F, cplx<T>* y, int nrhs,
                                    const double* E_rhs, const int* e_rhs, const int* sgn, const int* active) {
  if (nrhs <= 0) return hipSuccess;
  hipError_t err = launch_bloch_stencil_fused<T>(c, ph, F, y, nrhs, E_rhs, sgn, active);
  if (err != hipSuccess) return err;
  return launch_face_sigma<T>(c, F.pnew, y, nrhs, e_rhs, active);
}

template <typename T>
hipError_t launch_bloch_laplacian(iobm_ctx c, const BlochPhase& ph, double alpha, const cplx<T>* r, cplx<T>* z,
                                  int nrhs, const int* sgn, const int* active) {
  if (nrhs <= 0) return hipSuccess;
  const StencilArgs S = stencil_args(c, 16);
  const int rec = prof_start(c, IOBM_K_PRECOND_LAP);
  hipLaunchKernelGGL(k_bl_laplacian<T>, dim3(nrhs * S.nchunks), dim3(256), 0, c->stream, S, ph, exp(-alpha), r, z,
                     sgn, active);
  prof_stop(c, rec, 2.0 * nrhs * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bloch_dot(iobm_ctx c, const cplx<T>* u, const cplx<T>* v, int npairs, const int* pairs,
                            Partial* part, int nblk) {
  if (npairs <= 0) return hipSuccess;
  const int rec = prof_start(c, IOBM_K_BLOCH_VECTOR);
  hipLaunchKernelGGL(k_bl_dot<T>, dim3(npairs * nblk), dim3(256), 0, c->stream, u, v, c->g.npts, nblk, pairs, part);
  prof_stop(c, rec, 2.0 * npairs * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

hipError_t launch_bloch_scalars(iobm_ctx c, int mode, int npairs, const int* pairs, const Partial* pd,
                                const Partial* pn, int nblk, zd* rho, zd* alpha, zd* beta, double* rn2, int* flag) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bl_scalars, dim3((npairs + 63) / 64), dim3(64), 0, c->stream, mode, npairs, pairs, pd, pn,
                     nblk, rho, alpha, beta, rn2, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bloch_update(iobm_ctx c, cplx<T>* r, const cplx<T>* q, const zd* alpha, int nslots,
                               const int* active, Partial* pn, int nblk) {
  if (nslots <= 0) return hipSuccess;
  const int rec = prof_start(c, IOBM_K_BLOCH_VECTOR);
  hipLaunchKernelGGL(k_bl_update<T>, dim3(nslots * nblk), dim3(256), 0, c->stream, r, q, alpha, c->g.npts, nblk,
                     active, pn);
  // read r, q; write r
  prof_stop(c, rec, 3.0 * nslots * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bloch_settle(iobm_ctx c, zd* x, cplx<T>* d, const cplx<T>* p, const zd* alpha, int nslots,
                               const int* active, int nblk) {
  if (nslots <= 0) return hipSuccess;
  const int rec = prof_start(c, IOBM_K_BLOCH_VECTOR);
  hipLaunchKernelGGL(k_bl_settle<T>, dim3(nslots * nblk), dim3(256), 0, c->stream, x, d, p, alpha, c->g.npts, nblk,
                     active);
  // read and write x; read p; read and write d (complex64)
  prof_stop(c, rec, nslots * c->g.npts * (2.0 * sizeof(zd) + (d ? 3.0 : 1.0) * sizeof(cplx<T>)));
  return hipGetLastError();
}

#define IOBM_BLOCH_INST(T)                                                                                      \
  template hipError_t launch_bloch_apply_fused<T>(iobm_ctx, const BlochPhase&, const BlochFuse<T>&, cplx<T>*, int, \
                                                  const double*, const int*, const int*, const int*);          \
  template hipError_t launch_bloch_laplacian<T>(iobm_ctx, const BlochPhase&, double, const cplx<T>*, cplx<T>*,   \
                                                int, const int*, const int*);                                   \
  template hipError_t launch_bloch_dot<T>(iobm_ctx, const cplx<T>*, const cplx<T>*, int, const int*, Partial*,   \
                                          int);                                                                 \
  template hipError_t launch_bloch_update<T>(iobm_ctx, cplx<T>*, const cplx<T>*, const zd*, int, const int*,     \
                                             Partial*, int);                                                    \
  template hipError_t launch_bloch_settle<T>(iobm_ctx, zd*, cplx<T>*, const cplx<T>*, const zd*, int,          \
                                             const int*, int);
IOBM_BLOCH_INST(float)
IOBM_BLOCH_INST(double)
#undef IOBM_BLOCH_INST
