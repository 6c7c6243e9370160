// Block COCG kernels: the s x s Gram matrices of a group of right-hand sides
// that share one energy (the paper's incident waves of one energy, Sec. II),
// the s x s complex-symmetric solves for the block step lengths, and the
// block vector updates.
//
// Block COCG (the conjugate-gradient iteration the paper applies to its
// N_in incident waves, taken in block form with the bilinear product of the
// complex-symmetric A):
//   Q = A P;  alpha = (P^T Q)^-1 (R^T Z);  X += P alpha;  R -= Q alpha;
//   Z = M R;  beta = (R^T Z)_old^-1 (R^T Z)_new;  P = Z + P beta.
// A group's columns are a list of batch slots (cols[off .. off + s)), s <= 64.
// Every Gram entry is accumulated in FP64 (matrix cores, fp64 MFMA), and
// summed over point chunks in a fixed order.
#include "internal.h"

namespace {

typedef double acc4 __attribute__((ext_vector_type(4)));

constexpr int GRAM_PTS = 32;   // points per LDS chunk of the Gram kernel
constexpr int GRAM_WAVES = 4;  // wavefronts per Gram block

// G = U^T W for one group over the points of one block (a contiguous range),
// written as partials [group][block][a][b][4] packed per group (group g
// starts at poff[g] * nblk * 4 doubles, its s x s entries per block): the
// four real products (re re, re im, im re, im im) of columns a, b.  Tiles of 8 complex columns
// are 16 real rows: row 2a + c holds component c of column a.  MFMA
// 16x16x4 f64 operands (wave64): lane l holds A[row l % 16][k l / 16] and
// B[k l / 16][col l % 16]; accumulator entry v of lane l is D[row (l >> 4) +
// 4 v][col l % 16].  Only tiles ta <= tb are formed (the Grams are symmetric).
template <typename T>
__global__ void __launch_bounds__(64 * GRAM_WAVES) k_gram(const cplx<T>* __restrict__ U, const cplx<T>* __restrict__ W,
                                                          long long vol, const int* __restrict__ cols,
                                                          const int* __restrict__ goff, const int* __restrict__ gsize,
                                                          const int* __restrict__ poff, int nblk,
                                                          double* __restrict__ part) {
  __shared__ double su[64][GRAM_PTS][2];
  __shared__ double sw[64][GRAM_PTS][2];
  const int g = blockIdx.x / nblk;
  const int blk = blockIdx.x - g * nblk;
  const int s = gsize[g];
  const int* cg = cols + goff[g];
  const int nt = (s + 7) / 8;
  const int npairs = nt * (nt + 1) / 2;
  const long long per = ((vol + nblk - 1) / nblk + GRAM_PTS - 1) / GRAM_PTS * GRAM_PTS;
  const long long x0 = blk * per, x1 = min(vol, x0 + per);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // each wave owns the tile pairs wave, wave + GRAM_WAVES, ... (at most 9 of 36)
  acc4 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = acc4{0, 0, 0, 0};
  const int nrow = nt * 8;  // rows the tiles read (columns s..nrow-1 are zero)
  for (long long xc = x0; xc < x1; xc += GRAM_PTS) {
    __syncthreads();
    for (int e = threadIdx.x; e < nrow * GRAM_PTS; e += blockDim.x) {
      const int c = e / GRAM_PTS, p = e - c * GRAM_PTS;
      const long long x = xc + p;
      cplx<T> u = mk<T>(0, 0), w = mk<T>(0, 0);
      if (c < s && x < x1) {
        u = U[(long long)cg[c] * vol + x];
        w = W[(long long)cg[c] * vol + x];
      }
      su[c][p][0] = (double)u.re; su[c][p][1] = (double)u.im;
      sw[c][p][0] = (double)w.re; sw[c][p][1] = (double)w.im;
    }
    __syncthreads();
    const int r = lane & 15, k = lane >> 4;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int pr = wave + GRAM_WAVES * t;
      if (pr >= npairs) break;
      int ta = 0, rem = pr;
      while (rem >= nt - ta) { rem -= nt - ta; ++ta; }
      const int tb = ta + rem;
      const int a = ta * 8 + (r >> 1), ca = r & 1;
      const int b = tb * 8 + (r >> 1), cb = r & 1;
#pragma unroll
      for (int p = 0; p < GRAM_PTS; p += 4) {
        const double av = su[a][p + k][ca];
        const double bv = sw[b][p + k][cb];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
      }
    }
  }
  double* out = part + ((long long)poff[g] * nblk + (long long)blk * s * s) * 4;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int pr = wave + GRAM_WAVES * t;
    if (pr >= npairs) break;
    int ta = 0, rem = pr;
    while (rem >= nt - ta) { rem -= nt - ta; ++ta; }
    const int tb = ta + rem;
    const int col = lane & 15;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = (lane >> 4) + 4 * v;
      const int a = ta * 8 + (row >> 1), ca = row & 1;
      const int b = tb * 8 + (col >> 1), cb = col & 1;
      if (a < s && b < s) out[((long long)a * s + b) * 4 + ca * 2 + cb] = acc[t][v];
    }
  }
}

// Sum the block partials in block order into G[gid[group]][a][b] (complex,
// leading dimension 64): G = (re re - im im, re im + im re), formed from the
// pair with a <= b (the Grams U^T W of this solver are complex symmetric).
__global__ void __launch_bounds__(256) k_gram_reduce(const int* __restrict__ gsize, const int* __restrict__ gid,
                                                     const int* __restrict__ poff, int nblk,
                                                     const double* __restrict__ part, zd* __restrict__ G) {
  const int g = blockIdx.x;
  const int s = gsize[g];
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
    const int a = e / s, b = e - a * s;
    const int aa = min(a, b), bb = max(a, b);  // tile of aa is on or above the tile of bb
    double d[4] = {0, 0, 0, 0};
    for (int k = 0; k < nblk; ++k) {
      const double* p = part + ((long long)poff[g] * nblk + (long long)k * s * s + (long long)aa * s + bb) * 4;
      d[0] += p[0]; d[1] += p[1]; d[2] += p[2]; d[3] += p[3];
    }
    // u_aa^T w_bb = (re re - im im, re im + im re); entries below the diagonal
    // take their mirror image, so G is exactly symmetric
    G[(long long)gid[g] * 64 * 64 + (long long)a * 64 + b] = mk(d[0] - d[3], d[1] + d[2]);
  }
}

// Solve G X = Y for one group (s x s complex, FP64, leading dimension 64,
// matrices of group g at gid[g])
// by Gaussian elimination with partial pivoting on copies in the workspace;
// X overwrites Y's copy.  flag[g] = 1 when a pivot vanishes relative to the
// largest entry (the block has become rank deficient).
__global__ void __launch_bounds__(64) k_small_solve(const int* __restrict__ gsize, const int* __restrict__ gid,
                                                    const zd* __restrict__ Gin, const zd* __restrict__ Yin,
                                                    zd* __restrict__ Gw, zd* __restrict__ X, int* __restrict__ flag) {
  const int g = blockIdx.x;
  const int s = gsize[g];
  const long long o = (long long)gid[g] * 64 * 64;
  const zd* Gs = Gin + o;
  zd* A = Gw + o;
  zd* Y = X + o;
  __shared__ double red[64];
  __shared__ int piv;
  double amax = 0;
  for (int e = threadIdx.x; e < s * s; e += 64) {
    const int i = e / s, j = e - i * s;
    A[i * 64 + j] = Gs[i * 64 + j];
    Y[i * 64 + j] = Yin[o + i * 64 + j];
    amax = fmax(amax, sqrt(norm2(Gs[i * 64 + j])));
  }
  red[threadIdx.x] = amax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int i = 0; i < 64; ++i) m = fmax(m, red[i]);
    red[0] = m;
  }
  __syncthreads();
  const double scale = red[0];
  __syncthreads();
  bool bad = !(scale > 0) || !isfinite(scale);
  for (int k = 0; k < s && !bad; ++k) {
    if (threadIdx.x == 0) {
      int p = k;
      double best = -1;
      for (int i = k; i < s; ++i) {
        const double v = norm2(A[i * 64 + k]);
        if (v > best) { best = v; p = i; }
      }
      piv = p;
      red[0] = best;
    }
    __syncthreads();
    const int p = piv;
    if (!(sqrt(red[0]) > 1e-14 * scale)) { bad = true; break; }
    if (p != k)
      for (int j = threadIdx.x; j < s; j += 64) {
        zd t = A[k * 64 + j]; A[k * 64 + j] = A[p * 64 + j]; A[p * 64 + j] = t;
        zd u = Y[k * 64 + j]; Y[k * 64 + j] = Y[p * 64 + j]; Y[p * 64 + j] = u;
      }
    __syncthreads();
    const zd pk = A[k * 64 + k];
    const double n = norm2(pk);
    const zd inv = mk(pk.re / n, -pk.im / n);
    for (int i = k + 1; i < s; ++i) {
      const zd f = A[i * 64 + k] * inv;
      for (int j = threadIdx.x; j < s; j += 64) {
        if (j > k) A[i * 64 + j] = A[i * 64 + j] - f * A[k * 64 + j];
        Y[i * 64 + j] = Y[i * 64 + j] - f * Y[k * 64 + j];
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (!bad) {  // back substitution, one right-hand side column per thread
    for (int j = threadIdx.x; j < s; j += 64)
      for (int i = s - 1; i >= 0; --i) {
        zd acc = Y[i * 64 + j];
        for (int m = i + 1; m < s; ++m) acc = acc - A[i * 64 + m] * Y[m * 64 + j];
        const zd d = A[i * 64 + i];
        const double n = norm2(d);
        Y[i * 64 + j] = mk((acc.re * d.re + acc.im * d.im) / n, (acc.im * d.re - acc.re * d.im) / n);
      }
  }
  if (threadIdx.x == 0) flag[gid[g]] = bad ? 1 : 0;
  if (bad)
    for (int e = threadIdx.x; e < s * s; e += 64) Y[(e / s) * 64 + e % s] = mk(0.0, 0.0);
}

// Block update over the columns of each group, 64 points per block:
//   mode 0  Y[j] += sum_i X[i] C[i][j]
//   mode 1  Y[j] -= sum_i X[i] C[i][j], with the partials of |Y[j]|^2
//   mode 2  Y[j]  = Z[j] + sum_i X[i] C[i][j]
// X's columns at the block's points are staged in LDS; C (FP64, leading
// dimension 64) is applied in the iteration precision.  Y may be complex128
// (the solution) while X is complex64.
template <typename T, typename TY>
__global__ void __launch_bounds__(256) k_block_update(cplx<TY>* __restrict__ Y, const cplx<T>* __restrict__ X,
                                                      const cplx<T>* __restrict__ Z, const zd* __restrict__ C,
                                                      long long vol, const int* __restrict__ cols,
                                                      const int* __restrict__ goff, const int* __restrict__ gsize,
                                                      const int* __restrict__ gid, int nchunk, int mode,
                                                      Partial* __restrict__ n2part) {
  __shared__ cplx<T> sx[64][64];
  const int g = blockIdx.x / nchunk;
  const int ch = blockIdx.x - g * nchunk;
  const int s = gsize[g];
  const int* cg = cols + goff[g];
  const zd* Cg = C + (long long)gid[g] * 64 * 64;
  const int p = threadIdx.x & 63, jw = threadIdx.x >> 6;
  for (long long x0 = (long long)ch * 64; x0 < vol; x0 += (long long)nchunk * 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < s * 64; e += blockDim.x) {
      const int c = e >> 6, q = e & 63;
      sx[c][q] = x0 + q < vol ? X[(long long)cg[c] * vol + x0 + q] : mk<T>(0, 0);
    }
    __syncthreads();
    const long long x = x0 + p;
    if (x < vol)
      for (int j = jw; j < s; j += 4) {
        cplx<T> acc = mk<T>(0, 0);
        for (int i = 0; i < s; ++i) acc = cfma(sx[i][p], cvt<T>(Cg[i * 64 + j]), acc);
        cplx<TY>* yp = Y + (long long)cg[j] * vol + x;
        if (mode == 0) {
          const cplx<TY> y = *yp;
          *yp = mk<TY>(y.re + (TY)acc.re, y.im + (TY)acc.im);
        } else if (mode == 1) {
          const cplx<TY> y = *yp;
          const cplx<TY> v = mk<TY>(y.re - (TY)acc.re, y.im - (TY)acc.im);
          *yp = v;
        } else {
          const cplx<T> zv = Z[(long long)cg[j] * vol + x];
          *yp = mk<TY>((TY)(zv.re + acc.re), (TY)(zv.im + acc.im));
        }
      }
  }
  if (mode == 1 && n2part) {
    // |Y[j]|^2 partials: the points of this block, one wavefront per column
    // group j = jw, jw + 4, ...; re-read in the same order (fixed sums)
    for (int j = jw; j < s; j += 4) {
      double acc = 0;
      for (long long x0 = (long long)ch * 64; x0 < vol; x0 += (long long)nchunk * 64) {
        const long long x = x0 + p;
        if (x < vol) {
          const cplx<TY> y = Y[(long long)cg[j] * vol + x];
          acc += (double)y.re * y.re + (double)y.im * y.im;
        }
      }
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (p == 0) {
        Partial P;
        P.re = P.im = P.pad = 0;
        P.n2 = acc;
        n2part[(long long)cg[j] * nchunk + ch] = P;
      }
    }
  }
}

}  // namespace

// Gram matrices of the listed groups: G[gid[g]] = U^T W (FP64, leading
// dimension 64).  poff[g] = sum of s^2 over the groups listed before g (the
// packed partials take nblk * 4 * sum s^2 doubles).  (ncols = the listed
// columns in all groups, for the timing hook's byte count: read U and W once)
template <typename T>
hipError_t launch_gram(iobm_ctx c, const cplx<T>* U, const cplx<T>* W, int ngroups, const int* cols,
                       const int* goff, const int* gsize, const int* gid, const int* poff, double* part, int nblk,
                       zd* G, int ncols) {
  if (ngroups <= 0) return hipSuccess;
  const int rec = prof_start(c, IOBM_K_BLOCK_GRAM);
  hipLaunchKernelGGL(k_gram<T>, dim3(ngroups * nblk), dim3(64 * GRAM_WAVES), 0, c->stream, U, W, c->g.npts, cols,
                     goff, gsize, poff, nblk, part);
  hipLaunchKernelGGL(k_gram_reduce, dim3(ngroups), dim3(256), 0, c->stream, gsize, gid, poff, nblk, part, G);
  prof_stop(c, rec, 2.0 * ncols * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

hipError_t launch_small_solve(iobm_ctx c, int ngroups, const int* gsize, const int* gid, const zd* G, const zd* Y,
                              zd* Gw, zd* X, int* flag) {
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_solve, dim3(ngroups), dim3(64), 0, c->stream, gsize, gid, G, Y, Gw, X, flag);
  return hipGetLastError();
}

// (timing hook: read X, read and write Y (mode 2: read Z, write Y), and the
// second read of Y for the norms in mode 1)
template <typename T, typename TY>
hipError_t launch_block_update(iobm_ctx c, cplx<TY>* Y, const cplx<T>* X, const cplx<T>* Z, const zd* C, int ngroups,
                               const int* cols, const int* goff, const int* gsize, const int* gid, int nchunk,
                               int mode, Partial* n2part, int ncols) {
  if (ngroups <= 0) return hipSuccess;
  const int rec = prof_start(c, IOBM_K_BLOCK_UPDATE);
  hipLaunchKernelGGL((k_block_update<T, TY>), dim3(ngroups * nchunk), dim3(256), 0, c->stream, Y, X, Z, C,
                     c->g.npts, cols, goff, gsize, gid, nchunk, mode, n2part);
  const double bytes = sizeof(cplx<T>) + (mode == 2 ? sizeof(cplx<T>) + sizeof(cplx<TY>)
                                                    : (mode == 1 && n2part ? 3.0 : 2.0) * sizeof(cplx<TY>));
  prof_stop(c, rec, bytes * ncols * c->g.npts);
  return hipGetLastError();
}

template hipError_t launch_gram<float>(iobm_ctx, const zf*, const zf*, int, const int*, const int*, const int*,
                                       const int*, const int*, double*, int, zd*, int);
template hipError_t launch_gram<double>(iobm_ctx, const zd*, const zd*, int, const int*, const int*, const int*,
                                        const int*, const int*, double*, int, zd*, int);
template hipError_t launch_block_update<float, float>(iobm_ctx, zf*, const zf*, const zf*, const zd*, int,
                                                      const int*, const int*, const int*, const int*, int, int,
                                                      Partial*, int);
template hipError_t launch_block_update<double, double>(iobm_ctx, zd*, const zd*, const zd*, const zd*, int,
                                                        const int*, const int*, const int*, const int*, int, int,
                                                        Partial*, int);
