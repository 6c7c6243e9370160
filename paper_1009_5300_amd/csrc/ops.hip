// Volume kernels of libiobm: the IOBM operator, its two preconditioners,
// right-hand sides, FP64-accumulated Krylov reductions, vector updates and
// the scattering readout.
//
// Layout: a batch of right-hand sides is [rhs][z][y][x] interleaved complex
// (complex64 or complex128), x fastest.  Kernels that work on a subset of
// the batch take `active` (slot -> rhs id) and are launched over the slots.
#include "internal.h"

namespace {

__device__ __forceinline__ int rhs_of(const int* active, int slot) {
  return active ? active[slot] : slot;
}

// ------------------------------------------------------- reductions ---
// Per-rhs partial sums of the bilinear form a^T b (no conjugation, the COCG
// inner product for the complex-symmetric A) and of |a|^2, accumulated in
// FP64; one partial per block, combined in fixed order by k_finish2.
// block_reduce3 needs a block of whole wavefronts; the result is in thread 0.
__device__ __forceinline__ void block_reduce3(double& a, double& b, double& c) {
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

// Block sum of two values for a block of BLK threads that need not be whole
// wavefronts: staged through LDS, the first wavefront sums strided entries
// and then reduces across its lanes (a block smaller than a wavefront is
// summed by thread 0).  Result in thread 0.
template <int BLK>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double red[2][BLK];
  __syncthreads();
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  if constexpr (BLK < 64) {  // less than a wavefront: thread 0 sums in order
    if (threadIdx.x == 0) {
      double x = 0, y = 0;
      for (int i = 0; i < BLK; ++i) { x += red[0][i]; y += red[1][i]; }
      a = x;
      b = y;
    }
  } else if (threadIdx.x < 64) {
    double x = 0, y = 0;
    for (int i = threadIdx.x; i < BLK; i += 64) { x += red[0][i]; y += red[1][i]; }
    for (int off = 32; off > 0; off >>= 1) {
      x += __shfl_xor(x, off);
      y += __shfl_xor(y, off);
    }
    a = x;
    b = y;
  }
}

template <typename T> struct Real;
template <> struct Real<double> { static __device__ __forceinline__ double v(double x) { return x; } };
template <> struct Real<float> { static __device__ __forceinline__ float v(double x) { return (float)x; } };

template <typename T> __device__ __forceinline__ const T* potential(const double* Vd, const float* Vf);
template <> __device__ __forceinline__ const double* potential<double>(const double* Vd, const float*) { return Vd; }
template <> __device__ __forceinline__ const float* potential<float>(const double*, const float* Vf) { return Vf; }

// ------------------------------------------------------------ stencil ---
// y = (E - V) x - (H_kin) x on the truncated grid (Eqs. (1)-(4), (6)):
//   A x = (E - V + e0) x + sum_{mu, n=1..nf} w_{mu,n} [x(r + n e_mu) + x(r - n e_mu)],
//   e0 = (chat_0/2) sum_mu 1/h_mu^2,  w_{mu,n} = chat_n / (2 h_mu^2),
// lateral neighbours wrap (kappa = 0), z neighbours outside 0..nz-1 dropped.
// One block owns full lateral planes of one rhs over a chunk of planes.
// Operand and epilogue policies of the stencil kernels.  bind() selects the
// rhs, load(o) returns the operand at flat offset o of that rhs (load_raw and
// combine split it into the memory reads and the arithmetic, for prefetching
// lookahead planes ahead), center()
// sees the operand of each point the block owns, store() takes the operand
// and the stencil result of that point, and finish() runs once per block
// (every thread; it may synchronise the block).
template <typename T>
struct OpPlain {  // y = A_st x
  typedef cplx<T> Raw;
  static constexpr int lookahead = 2;
  static constexpr bool bloch = false;  // lateral couplings without bond phases
  const cplx<T>* x;
  cplx<T>* y;
  __device__ __forceinline__ void bind(int rhs, long long vol) { x += rhs * vol; y += rhs * vol; }
  __device__ __forceinline__ cplx<T> load(long long o) const { return x[o]; }
  __device__ __forceinline__ Raw load_raw(long long o, bool) const { return x[o]; }
  __device__ __forceinline__ cplx<T> combine(Raw r, bool ok) const { return ok ? r : mk<T>(0, 0); }
  __device__ __forceinline__ void side(const Raw&, long long, bool) {}
  __device__ __forceinline__ void center(long long, cplx<T>) {}
  __device__ __forceinline__ void center_at(long long, cplx<T>) {}
  __device__ __forceinline__ void store(int, long long o, cplx<T>, cplx<T> acc) { y[o] = acc; }
  __device__ __forceinline__ void finish(int, int, int) {}
};

// The number of z chunks of a launch depends on the batch size, so the
// chunk-0 block of each rhs zeroes the stencil slots past the last chunk.
__device__ __forceinline__ void clear_unused_slots(Partial* part, int rhs, int chunk, int nchunks) {
  if (chunk == 0 && (int)threadIdx.x < PQ_STENCIL_MAX - nchunks) {
    Partial Z;
    Z.re = Z.im = Z.n2 = Z.pad = 0;
    part[(long long)rhs * PQ_SLOTS + nchunks + threadIdx.x] = Z;
  }
}

// COCG direction update fused into the operator: the operand is
// p_new = z + beta p_old (p_old not read where beta = 0 and no update is
// pending), written to pnew for the block's own points; the block's partial
// of p_new^T y goes to part[rhs][chunk] (PQ_SLOTS per rhs).  With alpha set,
// the previous step's solution update d += alpha p_old is applied to the
// block's own points from the same p_old loads (skipped where alpha = 0,
// the first step after a restart).
template <typename T>
struct OpFuseP {
  struct Raw {
    cplx<T> z, p, d;
  };
  static constexpr int lookahead = sizeof(T) == 4 ? 2 : 1;
  static constexpr bool bloch = false;
  const cplx<T>* z;
  const cplx<T>* pold;
  const zd* beta;
  cplx<T>* pnew;
  cplx<T>* y;
  Partial* part;
  const zd* alpha;  // pending alpha per rhs, or nullptr
  cplx<T>* d;
  const int* dlive;  // per rhs: d holds data (else it counts as zero and is not read)
  const cplx<T>* psrc;
  const cplx<T>* dsrc;
  cplx<T> bt, at;
  bool use_b, use_p, use_d, live;
  double s_re, s_im;
  __device__ __forceinline__ void bind(int rhs, long long vol) {
    z += rhs * vol; pold += rhs * vol; pnew += rhs * vol; y += rhs * vol;
    bt = cvt<T>(beta[rhs]);
    at = alpha ? cvt<T>(alpha[rhs]) : mk<T>(0, 0);
    use_d = alpha && (alpha[rhs].re != 0 || alpha[rhs].im != 0);
    live = use_d && dlive[rhs] != 0;
    if (use_d) d += rhs * vol;
    use_b = bt.re != (T)0 || bt.im != (T)0;
    use_p = use_b || use_d;
    // where a stream is not needed its loads read z again: cache hits, not
    // another stream
    psrc = use_p ? pold : z;
    dsrc = live ? d : z;
    s_re = s_im = 0;
  }
  __device__ __forceinline__ cplx<T> load(long long o) const {
    cplx<T> v = z[o];
    if (use_b) v = v + bt * pold[o];
    return v;
  }
  __device__ __forceinline__ Raw load_raw(long long o, bool own) const {
    Raw r;
    r.z = z[o];
    r.p = psrc[o];
    r.d = (own ? dsrc : z)[o];
    return r;
  }
  __device__ __forceinline__ cplx<T> combine(const Raw& r, bool ok) const {
    return ok ? (use_b ? r.z + bt * r.p : r.z) : mk<T>(0, 0);
  }
  // a plane entering the window: the pending update of the block's own points
  __device__ __forceinline__ void side(const Raw& r, long long o, bool own) {
    if (use_d && own) d[o] = live ? r.d + at * r.p : at * r.p;
  }
  __device__ __forceinline__ void center(long long o, cplx<T> v) { pnew[o] = v; }
  // the cache-based kernel: the same at the centre point
  __device__ __forceinline__ void center_at(long long o, cplx<T> v) {
    pnew[o] = v;
    if (use_d) d[o] = live ? d[o] + at * pold[o] : at * pold[o];
  }
  __device__ __forceinline__ void store(int, long long o, cplx<T> c, cplx<T> acc) {
    y[o] = acc;
    s_re += (double)c.re * acc.re - (double)c.im * acc.im;
    s_im += (double)c.re * acc.im + (double)c.im * acc.re;
  }
  __device__ __forceinline__ void finish(int rhs, int chunk, int nchunks) {
    double dummy = 0;
    block_reduce3(s_re, s_im, dummy);
    if (threadIdx.x == 0) {
      Partial P;
      P.re = s_re; P.im = s_im; P.n2 = 0; P.pad = 0;
      part[(long long)rhs * PQ_SLOTS + chunk] = P;
    }
    clear_unused_slots(part, rhs, chunk, nchunks);
  }
};

// The phased stencil of the pair iteration at a lateral Bloch vector with the
// direction update fused, as OpFuseP does for the complex-symmetric
// iteration: the operand is p_new = z + beta p_old (p_old not read where
// beta = 0 and no update is pending), written to pnew for the block's own
// points, and the previous step's correction d += alpha p_old is applied to
// the own points from the same p_old loads (d is the FP64 solution itself
// in complex128).  beta and alpha are per pair (slot / 2).  Lateral
// couplings in the gauge u = exp(-i kappa.r) psi: the neighbour at +n
// along a direction enters with the weight times exp(i n kappa h), the one
// at -n with its conjugate; f[dir][n] holds weight x phase for the rhs at
// +kappa, and the rhs at -kappa (sgn < 0) take the conjugates.
template <typename T>
struct OpBlochFuse {
  // complex64 prefetches d with z and p; complex128 reads it when the plane
  // enters the window (its register queue would otherwise spill)
  static constexpr bool pre_d = sizeof(T) == sizeof(float);
  struct Raw {
    cplx<T> z, p, d;
  };
  static constexpr int lookahead = sizeof(T) == 4 ? 2 : 1;
  static constexpr bool bloch = true;
  const cplx<T>* z;
  const cplx<T>* pold;
  cplx<T>* pnew;
  cplx<T>* y;
  cplx<T>* d;
  const zd* beta;
  const zd* alpha;
  const int* sgn;
  cplx<T> f[2][4];
  const cplx<T>* psrc;
  cplx<T> bt, at;
  bool use_b, use_d;
  __device__ __forceinline__ void bind(int rhs, long long vol) {
    z += rhs * vol; pold += rhs * vol; pnew += rhs * vol; y += rhs * vol; d += rhs * vol;
    const zd b = beta[rhs >> 1], a = alpha[rhs >> 1];
    bt = cvt<T>(b);
    at = cvt<T>(a);
    use_b = b.re != 0 || b.im != 0;
    use_d = a.re != 0 || a.im != 0;
    psrc = (use_b || use_d) ? pold : z;
    if (sgn[rhs] < 0)
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int n = 1; n < 4; ++n) f[e][n] = conj(f[e][n]);
  }
  __device__ __forceinline__ cplx<T> load(long long o) const {
    cplx<T> v = z[o];
    if (use_b) v = v + bt * pold[o];
    return v;
  }
  __device__ __forceinline__ Raw load_raw(long long o, bool own) const {
    Raw r;
    r.z = z[o];
    r.p = psrc[o];
    if constexpr (pre_d) r.d = (own && use_d ? d : z)[o];
    return r;
  }
  __device__ __forceinline__ cplx<T> combine(const Raw& r, bool ok) const {
    return ok ? (use_b ? r.z + bt * r.p : r.z) : mk<T>(0, 0);
  }
  __device__ __forceinline__ void side(const Raw& r, long long o, bool own) {
    if (use_d && own) d[o] = (pre_d ? r.d : d[o]) + at * r.p;
  }
  __device__ __forceinline__ void center(long long o, cplx<T> v) { pnew[o] = v; }
  __device__ __forceinline__ void center_at(long long o, cplx<T> v) {
    pnew[o] = v;
    if (use_d) d[o] = d[o] + at * pold[o];
  }
  __device__ __forceinline__ void store(int, long long o, cplx<T>, cplx<T> acc) { y[o] = acc; }
  __device__ __forceinline__ void finish(int, int, int) {}
  __device__ __forceinline__ cplx<T> lat(int dir, int n, cplx<T> ap, cplx<T> am) const {
    return cfma(conj(f[dir][n]), am, f[dir][n] * ap);
  }
};

// FP64 residual of the refinement, r = b - A x, with b supported on the
// 2 nf electrode-face planes only (true of every right-hand side the solver
// builds).  Interior planes: r = -A_st x, stored in the iteration precision
// TR, with the block's partial of |r|^2 (FP64, from the complex128 values)
// in part[rhs][chunk].  Face planes: b - A_st x is kept in complex128 in
// rface for the electrode kernel, which adds Sigma x and finishes them.
template <typename TR>
struct OpRefresh {
  typedef zd Raw;
  static constexpr int lookahead = 1;
  static constexpr bool bloch = false;
  const zd* x;
  const zd* b;
  zd* rface;
  cplx<TR>* r;
  Partial* part;
  int nz, nf, nxy;
  double s_n2;
  __device__ __forceinline__ void bind(int rhs, long long vol) {
    x += rhs * vol; b += rhs * vol; rface += rhs * vol; r += rhs * vol;
    s_n2 = 0;
  }
  __device__ __forceinline__ zd load(long long o) const { return x[o]; }
  __device__ __forceinline__ Raw load_raw(long long o, bool) const { return x[o]; }
  __device__ __forceinline__ zd combine(Raw r, bool ok) const { return ok ? r : mk(0.0, 0.0); }
  __device__ __forceinline__ void side(const Raw&, long long, bool) {}
  __device__ __forceinline__ void center(long long, zd) {}
  __device__ __forceinline__ void center_at(long long, zd) {}
  __device__ __forceinline__ void store(int zz, long long o, zd, zd acc) {
    if (zz < nf || zz >= nz - nf) {
      rface[o] = b[o] - acc;
    } else {
      r[o] = cvt<TR>(-acc);
      s_n2 += acc.re * acc.re + acc.im * acc.im;
    }
  }
  __device__ __forceinline__ void finish(int rhs, int chunk, int nchunks) {
    double d0 = 0, d1 = 0;
    block_reduce3(s_n2, d0, d1);
    if (threadIdx.x == 0) {
      Partial P;
      P.re = 0; P.im = 0; P.n2 = s_n2; P.pad = 0;
      part[(long long)rhs * PQ_SLOTS + chunk] = P;
    }
    clear_unused_slots(part, rhs, chunk, nchunks);
  }
};

// The same residual at a lateral Bloch vector: the stencil in the gauge u
// with the lateral bond phases of OpBlochFuse (weights times phases in f,
// the rhs at -kappa, sgn < 0, taking the conjugates).
template <typename TR>
struct OpBlochRefresh : OpRefresh<TR> {
  static constexpr bool bloch = true;
  const int* sgn;
  zd f[2][4];
  __device__ __forceinline__ void bind(int rhs, long long vol) {
    OpRefresh<TR>::bind(rhs, vol);
    if (sgn[rhs] < 0)
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int n = 1; n < 4; ++n) f[e][n] = conj(f[e][n]);
  }
  __device__ __forceinline__ zd lat(int dir, int n, zd ap, zd am) const {
    return cfma(conj(f[dir][n]), am, f[dir][n] * ap);
  }
};

// Cache-based stencil (any plane size): one thread per point of a chunk of
// planes, every neighbour read from memory.
template <typename T, class Op>
__global__ void __launch_bounds__(256) k_apply(StencilArgs S, Op op, const T* __restrict__ V,
                                               const double* __restrict__ E_rhs,
                                               const int* __restrict__ active) {
  const int slot = blockIdx.x / S.nchunks;
  const int chunk = blockIdx.x - slot * S.nchunks;
  const int rhs = rhs_of(active, slot);
  op.bind(rhs, (long long)S.nxy * S.nz);
  const T diag0 = Real<T>::v(E_rhs[rhs] + S.e0);
  const int z0 = chunk * S.zchunk;
  const int z1 = min(S.nz, z0 + S.zchunk);
  T wx[4], wy[4], wz[4];
#pragma unroll
  for (int n = 1; n <= 3; ++n) { wx[n] = (T)S.wx[n]; wy[n] = (T)S.wy[n]; wz[n] = (T)S.wz[n]; }
  for (int z = z0; z < z1; ++z) {
    const long long zo = (long long)z * S.nxy;
    for (int p = threadIdx.x; p < S.nxy; p += blockDim.x) {
      const int j = p / S.nx;
      const int i = p - j * S.nx;
      const cplx<T> c0 = op.load(zo + p);
      op.center_at(zo + p, c0);
      const T d = diag0 - V[zo + p];
      cplx<T> acc = d * c0;
      for (int n = 1; n <= S.nf; ++n) {
        int ip = i + n; if (ip >= S.nx) ip -= S.nx;
        int im = i - n; if (im < 0) im += S.nx;
        int jp = j + n; if (jp >= S.ny) jp -= S.ny;
        int jm = j - n; if (jm < 0) jm += S.ny;
        if constexpr (Op::bloch) {
          acc = acc + op.lat(0, n, op.load(zo + j * S.nx + ip), op.load(zo + j * S.nx + im)) +
                op.lat(1, n, op.load(zo + jp * S.nx + i), op.load(zo + jm * S.nx + i));
        } else {
          cplx<T> sx = op.load(zo + j * S.nx + ip) + op.load(zo + j * S.nx + im);
          cplx<T> sy = op.load(zo + jp * S.nx + i) + op.load(zo + jm * S.nx + i);
          acc = acc + wx[n] * sx + wy[n] * sy;
        }
        cplx<T> sz = mk<T>(0, 0);
        if (z + n < S.nz) sz = sz + op.load(zo + (long long)n * S.nxy + p);
        if (z - n >= 0) sz = sz + op.load(zo - (long long)n * S.nxy + p);
        acc = acc + wz[n] * sz;
      }
      op.store(z, zo + p, c0, acc);
    }
  }
  op.finish(rhs, chunk, S.nchunks);
}

// 2.5D variant: a block owns all points of the lateral plane (up to MAXP per
// thread) of one rhs over a chunk of planes.  The current plane sits in LDS
// (double buffered, one barrier per plane) for the lateral neighbours; the
// z neighbours come from a per-thread register queue of 2 NF + 2 planes,
// which also prefetches the plane after the leading one.  Each operand
// element is read from memory once per chunk (plus 2 NF halo planes), each
// result written once.

// Largest block of each points-per-thread variant (planes up to 2304 points
// at any order, up to 4096 at nf = 1; larger planes take the cache-based
// kernel); the bound sets the compiler's register budget.
template <int MAXP>
struct A25 {
  static constexpr int max_threads = MAXP == 3 ? 768 : (MAXP == 4 ? 640 : 1024);
};

template <typename T, int NF, int MAXP, class Op>
__global__ void __launch_bounds__(A25<MAXP>::max_threads) k_apply25(StencilArgs S, Op op, const T* __restrict__ V,
                                                                    const double* __restrict__ E_rhs,
                                                                    const int* __restrict__ active) {
  typedef typename Op::Raw Raw;
  constexpr int W = 2 * NF + 1;  // planes of the z window
  constexpr int LA = Op::lookahead;
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);  // [2][nxy]
  const int nxy = S.nxy, nz = S.nz;
  const int slot = blockIdx.x / S.nchunks;
  const int chunk = blockIdx.x - slot * S.nchunks;
  const int rhs = rhs_of(active, slot);
  op.bind(rhs, (long long)nxy * nz);
  const T diag0 = Real<T>::v(E_rhs[rhs] + S.e0);
  const int z0 = chunk * S.zchunk;
  const int z1 = min(nz, z0 + S.zchunk);
  T wx[NF + 1], wy[NF + 1], wz[NF + 1];
#pragma unroll
  for (int n = 1; n <= NF; ++n) { wx[n] = (T)S.wx[n]; wy[n] = (T)S.wy[n]; wz[n] = (T)S.wz[n]; }
  // At step z: w[d][u] = operand(z - NF + d) at the thread's point u; pre[k][u]
  // holds the raw loads of plane z + NF + 1 + k, issued LA steps ahead and
  // combined into the window only when it advances, so that no step waits
  // on loads it has just issued.
  cplx<T> w[W][MAXP];
  Raw pre[LA][MAXP];
  T vq[2][MAXP];  // V(z), V(z + 1)
  // Loads are unconditional from clamped (always valid) addresses, and planes
  // outside 0..nz-1 or points past nxy are masked where the value is
  // combined: a load under a branch makes the compiler wait for it (and for
  // every load issued before it) at the branch's end.
  auto off = [&](int z, int u) -> long long {
    const int p = min((int)(threadIdx.x + u * blockDim.x), nxy - 1);
    return (long long)min(max(z, 0), nz - 1) * nxy + p;
  };
  auto valid = [&](int z, int u) -> bool {
    return (int)(threadIdx.x + u * blockDim.x) < nxy && z >= 0 && z < nz;
  };
  // the block's own points (the operator may update them when they enter
  // the window)
  auto own = [&](int z, int u) -> bool { return valid(z, u) && z >= z0 && z < z1; };
#pragma unroll
  for (int d = 0; d < W; ++d)
#pragma unroll
    for (int u = 0; u < MAXP; ++u) {
      const int zz = z0 - NF + d;
      const Raw r = op.load_raw(off(zz, u), own(zz, u));
      w[d][u] = op.combine(r, valid(zz, u));
      op.side(r, off(zz, u), own(zz, u));
    }
#pragma unroll
  for (int k = 0; k < LA; ++k)
#pragma unroll
    for (int u = 0; u < MAXP; ++u) pre[k][u] = op.load_raw(off(z0 + NF + 1 + k, u), own(z0 + NF + 1 + k, u));
#pragma unroll
  for (int u = 0; u < MAXP; ++u) vq[0][u] = V[off(z0, u)];
  for (int z = z0; z < z1; ++z) {
    const int b = (z - z0) & 1;
#pragma unroll
    for (int u = 0; u < MAXP; ++u) {
      const int p = threadIdx.x + u * blockDim.x;
      vq[1][u] = V[off(z + 1, u)];  // unused past the last plane
      if (p < nxy) {
        buf[b * nxy + p] = w[NF][u];
        op.center((long long)z * nxy + p, w[NF][u]);
      }
    }
    __syncthreads();
    const cplx<T>* pl = buf + b * nxy;
#pragma unroll
    for (int u = 0; u < MAXP; ++u) {
      const int p = threadIdx.x + u * blockDim.x;
      if (p < nxy) {
        const int j = p / S.nx;
        const int i = p - j * S.nx;
        cplx<T> acc = (diag0 - vq[0][u]) * w[NF][u];
#pragma unroll
        for (int n = 1; n <= NF; ++n) {
          int ip = i + n; if (ip >= S.nx) ip -= S.nx;
          int im = i - n; if (im < 0) im += S.nx;
          int jp = j + n; if (jp >= S.ny) jp -= S.ny;
          int jm = j - n; if (jm < 0) jm += S.ny;
          if constexpr (Op::bloch)
            acc = acc + op.lat(0, n, pl[j * S.nx + ip], pl[j * S.nx + im]) +
                  op.lat(1, n, pl[jp * S.nx + i], pl[jm * S.nx + i]) + wz[n] * (w[NF + n][u] + w[NF - n][u]);
          else
            acc = acc + wx[n] * (pl[j * S.nx + ip] + pl[j * S.nx + im]) +
                  wy[n] * (pl[jp * S.nx + i] + pl[jm * S.nx + i]) + wz[n] * (w[NF + n][u] + w[NF - n][u]);
        }
        op.store(z, (long long)z * nxy + p, w[NF][u], acc);
      }
    }
    // advance the window; issue the loads of plane z + NF + 1 + LA
#pragma unroll
    for (int u = 0; u < MAXP; ++u) {
#pragma unroll
      for (int d = 0; d < W - 1; ++d) w[d][u] = w[d + 1][u];
      w[W - 1][u] = op.combine(pre[0][u], valid(z + NF + 1, u));
      op.side(pre[0][u], off(z + NF + 1, u), own(z + NF + 1, u));
#pragma unroll
      for (int k = 0; k < LA - 1; ++k) pre[k][u] = pre[k + 1][u];
      pre[LA - 1][u] = op.load_raw(off(z + NF + 1 + LA, u), own(z + NF + 1 + LA, u));
      vq[0][u] = vq[1][u];
    }
  }
  op.finish(rhs, chunk, S.nchunks);
}

// Vector type for pairs of elements in global accesses (16 bytes: two
// complex64 or one complex128).
template <typename T> struct Pair;
template <> struct Pair<float> {
  typedef float4 type;
  static constexpr int n = 2;
  static __device__ __forceinline__ zf get(const float4& v, int k) { return k ? mk(v.z, v.w) : mk(v.x, v.y); }
  static __device__ __forceinline__ void set(float4& v, int k, zf c) {
    if (k) { v.z = c.re; v.w = c.im; } else { v.x = c.re; v.y = c.im; }
  }
};
template <> struct Pair<double> {
  typedef double2 type;
  static constexpr int n = 1;
  static __device__ __forceinline__ zd get(const double2& v, int) { return mk(v.x, v.y); }
  static __device__ __forceinline__ void set(double2& v, int, zd c) { v.x = c.re; v.y = c.im; }
};

// ----------------------------------------------------- electrode term ---
// y[boundary planes] -= Sigma x[boundary planes], applied in lateral
// momentum space (Eqs. (14)-(16)): FFT each of the nf planes, mix the planes
// of every mode with its nf x nf block, inverse FFT, scale by 1/Nxy.
// Block (slot, side); side 0 = left (planes 0..nf-1, reversed block),
// side 1 = right (planes nz-nf..nz-1).  With part set, the block's partial
// of x^T (its change of y) goes to part[rhs][pslot + side].  With rout set
// (the refinement residual), y holds b - A_st x on the faces and the block
// writes rout = y + Sigma x in precision TR and the partial of |rout|^2.
template <typename T, typename TR>
__global__ void k_boundary(FFTPlan2D plan, int nz, int nf, const cplx<T>* __restrict__ x,
                           cplx<T>* __restrict__ y, cplx<TR>* __restrict__ rout,
                           const cplx<T>* __restrict__ sig,
                           const int* __restrict__ e_rhs, const cplx<T>* __restrict__ twx,
                           const cplx<T>* __restrict__ twy, const int* __restrict__ active,
                           Partial* __restrict__ part, int np, int pslot) {
  extern __shared__ char smem_raw[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
  const int nxy = plan.x.n * plan.y.n;
  const int slot = blockIdx.x >> 1;
  const int side = blockIdx.x & 1;
  const int rhs = rhs_of(active, slot);
  const long long vol = (long long)nxy * nz;
  const cplx<T>* sg = sig + (long long)e_rhs[rhs] * nf * nf * nxy;  // [k][mode]
  cplx<T>* P[4];
  for (int k = 0; k <= nf; ++k) P[k] = buf + k * nxy;
  const int pbase = side ? nz - nf : 0;
  for (int k = 0; k < nf; ++k) {
    const cplx<T>* src = x + rhs * vol + (long long)(pbase + k) * nxy;
    for (int p = threadIdx.x; p < nxy; p += blockDim.x) P[k][p] = src[p];
    __syncthreads();
    cplx<T>* res = fft2d_lds(P[k], P[nf], plan, twx, twy, -1);
    if (res != P[k]) { cplx<T>* t = P[k]; P[k] = P[nf]; P[nf] = t; }
  }
  // mode mixing; plane k of the block <-> boundary-plane index i:
  // right: i = k;  left: i = nf-1-k with the reversed block, i.e. the same
  // matrix indexed by (nf-1-k, nf-1-l).
  const T inv = (T)(1.0 / nxy);
  for (int m = threadIdx.x; m < nxy; m += blockDim.x) {
    cplx<T> in[3], out[3];
    for (int k = 0; k < nf; ++k) in[k] = P[k][m];
    for (int k = 0; k < nf; ++k) {
      cplx<T> s = mk<T>(0, 0);
      const int ik = side ? k : nf - 1 - k;
      for (int l = 0; l < nf; ++l) {
        const int il = side ? l : nf - 1 - l;
        s = s + sg[(long long)(ik * nf + il) * nxy + m] * in[l];
      }
      out[k] = inv * s;
    }
    for (int k = 0; k < nf; ++k) P[k][m] = out[k];
  }
  __syncthreads();
  double s_re = 0, s_im = 0, s_n2 = 0;
  for (int k = 0; k < nf; ++k) {
    cplx<T>* res = fft2d_lds(P[k], P[nf], plan, twx, twy, +1);
    const long long po = rhs * vol + (long long)(pbase + k) * nxy;
    for (int p = threadIdx.x; p < nxy; p += blockDim.x) {
      const cplx<T> r = res[p];
      if (rout) {
        const cplx<T> v = y[po + p] + r;
        rout[po + p] = cvt<TR>(v);
        s_n2 += (double)v.re * v.re + (double)v.im * v.im;
      } else {
        y[po + p] = y[po + p] - r;
        if (part) {  // x^T (y change) = -x^T Sigma x on this face
          const cplx<T> c = x[po + p];
          s_re -= (double)c.re * r.re - (double)c.im * r.im;
          s_im -= (double)c.re * r.im + (double)c.im * r.re;
        }
      }
    }
    __syncthreads();
  }
  if (part) {
    block_reduce3(s_re, s_im, s_n2);
    if (threadIdx.x == 0) {
      Partial Pp;
      Pp.re = s_re; Pp.im = s_im; Pp.n2 = s_n2; Pp.pad = 0;
      part[(long long)rhs * np + pslot + side] = Pp;
    }
  }
}

// Square planes (N x N, N in the register-FFT list): the NF face planes of
// one side sit in LDS (padded rows); N threads per plane transform its rows
// and then its columns in registers, both ways.  Same contract as
// k_boundary.  Block partials are staged in LDS and summed by thread 0 in
// thread order (blocks can be smaller than a wavefront).
template <typename T, typename TR, int N, int NF>
__global__ void __launch_bounds__(N * NF) k_boundary_reg(int nz, const cplx<T>* __restrict__ x,
                                                        cplx<T>* __restrict__ y, cplx<TR>* __restrict__ rout,
                                                        const cplx<T>* __restrict__ sig,
                                                        const int* __restrict__ e_rhs,
                                                        const cplx<T>* __restrict__ tw,
                                                        const int* __restrict__ active,
                                                        Partial* __restrict__ part, int np, int pslot) {
  constexpr int NN = N * N, BLK = N * NF;
  typedef typename Pair<T>::type VT;
  constexpr int PE = Pair<T>::n;              // elements per vector access
  constexpr int NV = NF * NN / PE;            // vector accesses of the nf planes
  constexpr int EPT = (NV + BLK - 1) / BLK;   // per thread
  constexpr int MPT = (NN + BLK - 1) / BLK;   // modes per thread
  // loads are issued in batches, each batch in flight at once: the kernel
  // has one short block per state and side, so a load waited on one at a
  // time would expose its latency once per element
  constexpr int B1 = 12, B5 = 8;
  constexpr int B3 = NF == 1 ? 24 : (NF == 2 ? 6 : 2);
  __shared__ cplx<T> sm[NF][N][N + 1];
  __shared__ double red[3][BLK];
  const int slot = blockIdx.x >> 1;
  const int side = blockIdx.x & 1;
  const int rhs = rhs_of(active, slot);
  const cplx<T>* sg = sig + (long long)e_rhs[rhs] * NF * NF * NN;  // [k][mode]
  const int pbase = side ? nz - NF : 0;
  const long long off = (long long)rhs * NN * nz + (long long)pbase * NN;  // NF consecutive planes
  auto at = [&](int el) -> cplx<T>& {
    const int kk = el / NN, e = el - kk * NN;
    return sm[kk][e / N][e % N];
  };
#pragma unroll
  for (int b0 = 0; b0 < EPT; b0 += B1) {
    VT buf[B1];
#pragma unroll
    for (int e = 0; e < B1; ++e) {
      const int v = threadIdx.x + (b0 + e) * BLK;
      if (b0 + e < EPT && v < NV) buf[e] = reinterpret_cast<const VT*>(x + off)[v];
    }
#pragma unroll
    for (int e = 0; e < B1; ++e) {
      const int v = threadIdx.x + (b0 + e) * BLK;
      if (b0 + e < EPT && v < NV)
#pragma unroll
        for (int k = 0; k < PE; ++k) at(v * PE + k) = Pair<T>::get(buf[e], k);
    }
  }
  __syncthreads();
  const int k = threadIdx.x / N, li = threadIdx.x - k * N;
  cplx<T> v[N];
  auto rows_cols = [&](int sign) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = sm[k][li][i];
    reg_fft<T, N>(v, tw, sign);
#pragma unroll
    for (int i = 0; i < N; ++i) sm[k][li][i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = sm[k][i][li];
    reg_fft<T, N>(v, tw, sign);
#pragma unroll
    for (int i = 0; i < N; ++i) sm[k][i][li] = v[i];
    __syncthreads();
  };
  rows_cols(-1);
  // mode mixing, mode m = ky N + kx at sm[.][ky][kx]; plane k <-> boundary
  // index i as in k_boundary
  const T inv = (T)(1.0 / NN);
#pragma unroll
  for (int j0 = 0; j0 < MPT; j0 += B3) {
    cplx<T> sv[B3][NF * NF];
#pragma unroll
    for (int jj = 0; jj < B3; ++jj) {
      const int m = threadIdx.x + (j0 + jj) * BLK;
      // entry (kk, l) of the block in plane order (the left side reverses
      // the planes), so that the register array is indexed statically
      if (j0 + jj < MPT && m < NN)
#pragma unroll
        for (int kk = 0; kk < NF; ++kk)
#pragma unroll
          for (int l = 0; l < NF; ++l) {
            const int ik = side ? kk : NF - 1 - kk, il = side ? l : NF - 1 - l;
            sv[jj][kk * NF + l] = sg[(ik * NF + il) * NN + m];
          }
    }
#pragma unroll
    for (int jj = 0; jj < B3; ++jj) {
      const int m = threadIdx.x + (j0 + jj) * BLK;
      if (j0 + jj < MPT && m < NN) {
        const int r = m / N, cc = m - r * N;
        cplx<T> in[NF];
#pragma unroll
        for (int l = 0; l < NF; ++l) in[l] = sm[l][r][cc];
#pragma unroll
        for (int kk = 0; kk < NF; ++kk) {
          cplx<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int l = 0; l < NF; ++l) acc = acc + sv[jj][kk * NF + l] * in[l];
          sm[kk][r][cc] = inv * acc;
        }
      }
    }
  }
  __syncthreads();
  rows_cols(+1);
  double s_re = 0, s_im = 0, s_n2 = 0;
#pragma unroll
  for (int b0 = 0; b0 < EPT; b0 += B5) {
    VT yv[B5], xv[B5];
#pragma unroll
    for (int e = 0; e < B5; ++e) {
      const int vv = threadIdx.x + (b0 + e) * BLK;
      if (b0 + e < EPT && vv < NV) {
        yv[e] = reinterpret_cast<const VT*>(y + off)[vv];
        if (part && !rout) xv[e] = reinterpret_cast<const VT*>(x + off)[vv];
      }
    }
#pragma unroll
    for (int e = 0; e < B5; ++e) {
      const int vv = threadIdx.x + (b0 + e) * BLK;
      if (b0 + e < EPT && vv < NV) {
#pragma unroll
        for (int kq = 0; kq < PE; ++kq) {
          const cplx<T> res = at(vv * PE + kq);
          const cplx<T> yc = Pair<T>::get(yv[e], kq);
          if (rout) {
            const cplx<T> val = yc + res;
            rout[off + vv * PE + kq] = cvt<TR>(val);
            s_n2 += (double)val.re * val.re + (double)val.im * val.im;
          } else {
            Pair<T>::set(yv[e], kq, yc - res);
            if (part) {
              const cplx<T> xc = Pair<T>::get(xv[e], kq);
              s_re -= (double)xc.re * res.re - (double)xc.im * res.im;
              s_im -= (double)xc.re * res.im + (double)xc.im * res.re;
            }
          }
        }
        if (!rout) reinterpret_cast<VT*>(y + off)[vv] = yv[e];
      }
    }
  }
  if (part) {
    red[0][threadIdx.x] = s_re;
    red[1][threadIdx.x] = s_im;
    red[2][threadIdx.x] = s_n2;
    __syncthreads();
    if (threadIdx.x == 0) {
      Partial P;
      P.re = P.im = P.n2 = P.pad = 0;
      for (int t = 0; t < BLK; ++t) { P.re += red[0][t]; P.im += red[1][t]; P.n2 += red[2][t]; }
      part[(long long)rhs * np + pslot + side] = P;
    }
  }
}

// ----------------------------------------------- Eq. (17) preconditioner ---
// z = C0 r + C1 sum over the six face neighbours, C0 = 1, C1 = exp(-alpha);
// lateral neighbours wrap, z neighbours outside the region are zero.
template <typename T>
__global__ void __launch_bounds__(256) k_precond_lap(StencilArgs S, T c1, const cplx<T>* __restrict__ r,
                                                     cplx<T>* __restrict__ z,
                                                     const int* __restrict__ active,
                                                     Partial* __restrict__ dpart) {
  const int slot = blockIdx.x / S.nchunks;
  const int chunk = blockIdx.x - slot * S.nchunks;
  const int rhs = rhs_of(active, slot);
  const long long vol = (long long)S.nxy * S.nz;
  const cplx<T>* rr = r + rhs * vol;
  cplx<T>* zr = z + rhs * vol;
  const int z0 = chunk * S.zchunk;
  const int z1 = min(S.nz, z0 + S.zchunk);
  double s_re = 0, s_im = 0;
  for (int k = z0; k < z1; ++k) {
    const cplx<T>* rp = rr + (long long)k * S.nxy;
    for (int p = threadIdx.x; p < S.nxy; p += blockDim.x) {
      const int j = p / S.nx;
      const int i = p - j * S.nx;
      int ip = i + 1; if (ip >= S.nx) ip -= S.nx;
      int im = i - 1; if (im < 0) im += S.nx;
      int jp = j + 1; if (jp >= S.ny) jp -= S.ny;
      int jm = j - 1; if (jm < 0) jm += S.ny;
      cplx<T> s = rp[j * S.nx + ip] + rp[j * S.nx + im] + rp[jp * S.nx + i] + rp[jm * S.nx + i];
      if (k + 1 < S.nz) s = s + rp[S.nxy + p];
      if (k > 0) s = s + rp[-S.nxy + p];
      const cplx<T> c = rp[p], v = c + c1 * s;
      zr[(long long)k * S.nxy + p] = v;
      s_re += (double)c.re * v.re - (double)c.im * v.im;
      s_im += (double)c.re * v.im + (double)c.im * v.re;
    }
  }
  if (dpart) {
    double dummy = 0;
    block_reduce3(s_re, s_im, dummy);
    if (threadIdx.x == 0) {
      Partial P;
      P.re = s_re; P.im = s_im; P.n2 = 0; P.pad = 0;
      dpart[(long long)rhs * S.nchunks + chunk] = P;
    }
  }
}

// ------------------------------------------------- Jacobi preconditioner ---
// z = r / a, a = diag A(E) = E - V + e0 - (nonlocal diagonal) - (diagonal of
// the real-space self-energy on the 2 nf face planes: the mean over the
// lateral modes of the nf x nf blocks' diagonal, Eq. (11)).  Per-rhs
// partials of r^T z, one per block of a contiguous chunk.
template <typename T>
__global__ void __launch_bounds__(256) k_precond_jacobi(const cplx<T>* __restrict__ r, cplx<T>* __restrict__ z,
                                                        const double* __restrict__ V, const double* __restrict__ kbd,
                                                        const zd* __restrict__ sdiag, const int* __restrict__ e_rhs,
                                                        const double* __restrict__ E_rhs, double e0, int nz, int nf,
                                                        int nxy, int nblk, const int* __restrict__ active,
                                                        Partial* __restrict__ dpart) {
  const int slot = blockIdx.x / nblk;
  const int blk = blockIdx.x - slot * nblk;
  const int rhs = rhs_of(active, slot);
  const long long vol = (long long)nxy * nz;
  const long long per = (vol + nblk - 1) / nblk;
  const long long i0 = blk * per, i1 = min(vol, i0 + per);
  const double d0 = E_rhs[rhs] + e0;
  const zd* sd = sdiag + (long long)e_rhs[rhs] * nf;
  double s_re = 0, s_im = 0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const int k = (int)(i / nxy);
    zd a = mk(d0 - V[i] - (kbd ? kbd[i] : 0.0), 0.0);
    if (k < nf) a = a - sd[nf - 1 - k];               // left face: reversed plane order
    else if (k >= nz - nf) a = a - sd[k - (nz - nf)];  // right face
    const double n = a.re * a.re + a.im * a.im;
    const zd inv = mk(a.re / n, -a.im / n);
    const cplx<T> c = r[rhs * vol + i];
    const cplx<T> v = cvt<T>(inv) * c;
    z[rhs * vol + i] = v;
    s_re += (double)c.re * v.re - (double)c.im * v.im;
    s_im += (double)c.re * v.im + (double)c.im * v.re;
  }
  if (dpart) {
    double dummy = 0;
    block_reduce3(s_re, s_im, dummy);
    if (threadIdx.x == 0) {
      Partial P;
      P.re = s_re; P.im = s_im; P.n2 = 0; P.pad = 0;
      dpart[(long long)rhs * nblk + blk] = P;
    }
  }
}

// Diagonal of the right self-energy in real space per energy and face plane
// i: (1/Nxy) sum over the lateral modes of Sigma~_nu[i][i], summed in a fixed
// order (one block per entry).
__global__ void __launch_bounds__(256) k_sigma_diag(const zd* __restrict__ sig, int nxy, int nf, zd* __restrict__ sdiag) {
  const int e = blockIdx.x / nf, i = blockIdx.x - e * nf;
  const zd* row = sig + ((long long)e * nf * nf + i * nf + i) * nxy;
  double re = 0, im = 0, dummy = 0;
  for (int m = threadIdx.x; m < nxy; m += blockDim.x) {
    re += row[m].re;
    im += row[m].im;
  }
  block_reduce3(re, im, dummy);
  if (threadIdx.x == 0) sdiag[blockIdx.x] = mk(re / nxy, im / nxy);
}

// ------------------------------------------ lateral-Fourier preconditioner ---
// z = (E - H_0 - Sigma_L - Sigma_R)^-1 r, the exact inverse of the operator
// of the flat (V = 0) wire.  It is diagonal in the lateral modes (Eq. (16));
// along z each mode's inverse is the lead Green's function G(z - z'), which
// obeys the outgoing recurrence, so it is applied as a causal plus an
// anti-causal order-nf recursive filter (coefficients from the mode setup).
// Three passes, each with ample parallelism:
//   1. k_fft_planes: forward 2D FFT of every plane (one block per plane),
//   2. k_zfilter: per mode, the two recursions along z on an LDS tile of
//      [nz][MB] modes of one rhs,
//   3. k_fft_planes: inverse 2D FFT in place, scaled by 1/Nxy.

// Batched 2D FFT of the planes of the active rhs; block = (slot, plane).
template <typename T>
__global__ void __launch_bounds__(256) k_fft_planes(FFTPlan2D plan, int nz, const cplx<T>* in,
                                                    cplx<T>* out, const cplx<T>* __restrict__ twx,
                                                    const cplx<T>* __restrict__ twy, int sign, T scale,
                                                    const int* __restrict__ active,
                                                    const cplx<T>* __restrict__ dvec,
                                                    Partial* __restrict__ dpart) {
  extern __shared__ char smem_raw[];
  cplx<T>* bufA = reinterpret_cast<cplx<T>*>(smem_raw);
  const int nxy = plan.x.n * plan.y.n;
  cplx<T>* bufB = bufA + nxy;
  const int slot = blockIdx.x / nz;
  const int z = blockIdx.x - slot * nz;
  const int rhs = rhs_of(active, slot);
  const long long off = (long long)rhs * nxy * nz + (long long)z * nxy;
  for (int p = threadIdx.x; p < nxy; p += blockDim.x) bufA[p] = in[off + p];
  __syncthreads();
  cplx<T>* res = fft2d_lds(bufA, bufB, plan, twx, twy, sign);
  double a = 0, b = 0, dummy = 0;
  for (int p = threadIdx.x; p < nxy; p += blockDim.x) {
    const cplx<T> v = scale * res[p];
    out[off + p] = v;
    if (dpart) {
      const cplx<T> d = dvec[off + p];
      a += (double)v.re * d.re - (double)v.im * d.im;
      b += (double)v.re * d.im + (double)v.im * d.re;
    }
  }
  if (dpart) {
    block_reduce3(a, b, dummy);
    if (threadIdx.x == 0) {
      Partial P;
      P.re = a; P.im = b; P.n2 = 0; P.pad = 0;
      dpart[(long long)rhs * nz + z] = P;
    }
  }
}

// Square planes (N x N, N in a fixed list): each thread transforms one row
// and then one column held in registers; the plane goes through LDS once
// (padded rows, N + 1, against bank conflicts).  PPB planes per block.  The
// global loads and stores move pairs of elements (16 bytes for complex64)
// and every thread issues all of its loads before the first LDS store, so
// that the few threads of a block keep many requests in flight.

// With mvec and dpart set (the inverse transform of the preconditioner),
// the block also writes, per plane, the partial of the bilinear form
// sum_x r(x) out(x), taken in mode space by Parseval:
//   sum_x r(x) out(x) = scale * sum_k R(-k) in(k),   R = forward FFT of r = mvec,
// from loads issued together with those of the input (a real-space dot
// would read r after the transforms, with its latency exposed).
// With MODE = FFT_UPDATE (the forward transform of the preconditioner in the
// COCG step), the residual is kept in lateral mode space, R = FFT(r): the
// block transforms in = q and updates out = R in place, R -= alpha FFT(q),
// and writes the per-plane partials of |r|^2 = |R|^2 / Nxy (Parseval) to
// dpart[rhs][z].  The real-space r is neither read nor written, and the
// transform of the preconditioner comes with the update.
enum { FFT_PLAIN = 0, FFT_DOT = 1, FFT_UPDATE = 2 };

// Threads per row of the register FFT: complex128 rows of 24 points and more
// take two threads, each holding half a row (a whole 48-point complex128 row
// and the transform's scratch exceed the register file and went to scratch
// memory); each transforms half the samples (even or odd) and the pair
// combines by one radix-2 step, exchanging values between adjacent lanes.
template <typename T, int N>
constexpr int fft_split() { return (sizeof(T) == 8 && N >= 24) ? 2 : 1; }

// One row (or column) of the plane in LDS, elements at a[i * stride],
// i < N, transformed in place by the SPLIT threads that own it (half = the
// thread's index in the pair); tw = exp(-2 pi i k / N), tw2 = exp(-2 pi i k
// / (N/2)).  The pair are adjacent lanes of one wavefront.
template <typename T, int N, int SPLIT>
__device__ __forceinline__ void lds_line_fft(cplx<T>* a, int stride, int half, const cplx<T>* tw,
                                             const cplx<T>* tw2, int sign, T scale) {
  if constexpr (SPLIT == 1) {
    cplx<T> v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = a[i * stride];
    reg_fft<T, N>(v, tw, sign);
#pragma unroll
    for (int i = 0; i < N; ++i) a[i * stride] = scale * v[i];
  } else {
    constexpr int M = N / 2;
    cplx<T> v[M];
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = a[(2 * m + half) * stride];  // even (half 0) or odd samples
    reg_fft<T, M>(v, tw2, sign);
    // X[k] = E[k] + w^k O[k], X[k + M] = E[k] - w^k O[k]; half 0 holds E and
    // writes X[k], half 1 holds O and writes X[k + M]
#pragma unroll
    for (int k = 0; k < M; ++k) {
      cplx<T> o;
      o.re = __shfl_xor(v[k].re, 1);
      o.im = __shfl_xor(v[k].im, 1);
      const cplx<T> e = half ? o : v[k];
      const cplx<T> t = twid(tw, k, sign) * (half ? v[k] : o);
      a[(k + half * M) * stride] = scale * (half ? e - t : e + t);
    }
  }
}

template <typename T, int N, int PPB, int MODE>
__global__ void __launch_bounds__((fft_split<T, N>() * N * PPB))
    k_fft_planes_reg(int nz, int nplanes, const cplx<T>* in, cplx<T>* out,
                                                           const cplx<T>* __restrict__ tw, int sign, T scale,
                                                           const int* __restrict__ active,
                                                           const cplx<T>* __restrict__ mvec,
                                                           Partial* __restrict__ dpart, FftUpd<T> U) {
  constexpr bool DOT = MODE == FFT_DOT;
  typedef typename Pair<T>::type VT;
  constexpr int PE = Pair<T>::n;          // elements per vector access
  constexpr int NN = N * N;
  constexpr int NV = PPB * NN / PE;       // vector accesses per block
  constexpr int SPLIT = fft_split<T, N>();
  constexpr int BLK = SPLIT * N * PPB;
  constexpr int EPT = (NV + BLK - 1) / BLK;
  __shared__ cplx<T> sm[PPB][N][N + 1];
  __shared__ cplx<T> tw2[N / 2 + 1];  // exp(-2 pi i k / (N/2)) for the split transform
  if (SPLIT > 1)
    for (int k = threadIdx.x; k < N / 2; k += BLK) tw2[k] = tw[2 * k];
  const long long vol = (long long)NN * nz;
  const int g0 = blockIdx.x * PPB;
  long long poff[PPB];
  bool pok[PPB];
  int prhs[PPB];
#pragma unroll
  for (int q = 0; q < PPB; ++q) {
    const int gp = g0 + q;
    pok[q] = gp < nplanes;
    const int slot = pok[q] ? gp / nz : 0, z = pok[q] ? gp - slot * nz : 0;
    prhs[q] = rhs_of(active, slot);
    poff[q] = (long long)prhs[q] * vol + (long long)z * NN;
  }
  VT buf[EPT];
  cplx<T> al[PPB];  // alpha of each plane's rhs (FFT_UPDATE)
#pragma unroll
  for (int q = 0; q < PPB; ++q) al[q] = (MODE == FFT_UPDATE && pok[q]) ? cvt<T>(U.alpha[prhs[q]]) : mk<T>(0, 0);
  double ds_re[PPB], ds_im[PPB];
#pragma unroll
  for (int q = 0; q < PPB; ++q) ds_re[q] = ds_im[q] = 0;
  if constexpr (DOT) {
    // R and the first half of the input in flight together, R staged in LDS,
    // then the second half: at most one and a half planes in registers
    constexpr int H = EPT / 2;
    VT mb[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int v = threadIdx.x + e * BLK;
      const int q = v / (NN / PE), w = v - q * (NN / PE);
      if (v < NV && pok[q]) mb[e] = reinterpret_cast<const VT*>(mvec + poff[q])[w];
    }
#pragma unroll
    for (int e = 0; e < H; ++e) {
      const int v = threadIdx.x + e * BLK;
      const int q = v / (NN / PE), w = v - q * (NN / PE);
      if (v < NV && pok[q]) buf[e] = reinterpret_cast<const VT*>(in + poff[q])[w];
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {  // stage R in LDS
      const int v = threadIdx.x + e * BLK;
      const int q = v / (NN / PE), w = v - q * (NN / PE);
      if (v < NV) {
#pragma unroll
        for (int k = 0; k < PE; ++k) {
          const int el = w * PE + k;
          sm[q][el / N][el % N] = Pair<T>::get(mb[e], k);
        }
      }
    }
#pragma unroll
    for (int e = H; e < EPT; ++e) {
      const int v = threadIdx.x + e * BLK;
      const int q = v / (NN / PE), w = v - q * (NN / PE);
      if (v < NV && pok[q]) buf[e] = reinterpret_cast<const VT*>(in + poff[q])[w];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {  // sum_k R(-k) in(k), mode k = (ky, kx) at row ky, column kx
      const int v = threadIdx.x + e * BLK;
      const int q = v / (NN / PE), w = v - q * (NN / PE);
      if (v < NV && pok[q]) {
#pragma unroll
        for (int k = 0; k < PE; ++k) {
          const int el = w * PE + k;
          const int ky = el / N, kx = el % N;
          const cplx<T> rm = sm[q][(N - ky) % N][(N - kx) % N];
          const cplx<T> ck = Pair<T>::get(buf[e], k);
#pragma unroll
          for (int qq = 0; qq < PPB; ++qq)
            if (qq == q) {
              ds_re[qq] += (double)ck.re * rm.re - (double)ck.im * rm.im;
              ds_im[qq] += (double)ck.re * rm.im + (double)ck.im * rm.re;
            }
        }
      }
    }
    __syncthreads();
  } else if constexpr (MODE == FFT_UPDATE) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int v = threadIdx.x + e * BLK;
      const int q = v / (NN / PE), w = v - q * (NN / PE);
      if (v < NV && pok[q]) buf[e] = reinterpret_cast<const VT*>(in + poff[q])[w];
    }
  } else {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int v = threadIdx.x + e * BLK;
      const int q = v / (NN / PE), w = v - q * (NN / PE);
      if (v < NV && pok[q]) buf[e] = reinterpret_cast<const VT*>(in + poff[q])[w];
    }
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int v = threadIdx.x + e * BLK;
    const int q = v / (NN / PE), w = v - q * (NN / PE);
    if (v < NV) {
#pragma unroll
      for (int k = 0; k < PE; ++k) {
        const int el = w * PE + k;
        sm[q][el / N][el % N] = Pair<T>::get(buf[e], k);
      }
    }
  }
  __syncthreads();
  const int pl = threadIdx.x / (SPLIT * N);
  const int li = (threadIdx.x - pl * SPLIT * N) / SPLIT, half = threadIdx.x % SPLIT;
  lds_line_fft<T, N, SPLIT>(&sm[pl][li][0], 1, half, tw, tw2, sign, (T)1);        // row li
  __syncthreads();
  lds_line_fft<T, N, SPLIT>(&sm[pl][0][li], N + 1, half, tw, tw2, sign, scale);  // column li
  __syncthreads();
  if constexpr (MODE == FFT_UPDATE) {
    // R -= alpha FFT(q), the old R loaded in two batches
    constexpr int H = (EPT + 1) / 2;
#pragma unroll
    for (int b0 = 0; b0 < EPT; b0 += H) {
      VT ro[H];
#pragma unroll
      for (int e = 0; e < H; ++e) {
        const int vv = threadIdx.x + (b0 + e) * BLK;
        const int q = vv / (NN / PE), w = vv - q * (NN / PE);
        if (b0 + e < EPT && vv < NV && pok[q]) ro[e] = reinterpret_cast<const VT*>(out + poff[q])[w];
      }
#pragma unroll
      for (int e = 0; e < H; ++e) {
        const int vv = threadIdx.x + (b0 + e) * BLK;
        const int q = vv / (NN / PE), w = vv - q * (NN / PE);
        if (b0 + e < EPT && vv < NV && pok[q]) {
#pragma unroll
          for (int k = 0; k < PE; ++k) {
            const int el = w * PE + k;
#pragma unroll
            for (int qq = 0; qq < PPB; ++qq)
              if (qq == q) {
                const cplx<T> ck = Pair<T>::get(ro[e], k) - al[qq] * sm[q][el / N][el % N];
                Pair<T>::set(ro[e], k, ck);
                ds_re[qq] += (double)ck.re * ck.re + (double)ck.im * ck.im;
              }
          }
          reinterpret_cast<VT*>(out + poff[q])[w] = ro[e];
        }
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int vv = threadIdx.x + e * BLK;
      const int q = vv / (NN / PE), w = vv - q * (NN / PE);
      if (vv < NV && pok[q]) {
        VT o;
#pragma unroll
        for (int k = 0; k < PE; ++k) {
          const int el = w * PE + k;
          Pair<T>::set(o, k, sm[q][el / N][el % N]);
        }
        reinterpret_cast<VT*>(out + poff[q])[w] = o;
      }
    }
  }
  if constexpr (MODE != FFT_PLAIN) {
#pragma unroll
    for (int q = 0; q < PPB; ++q) {
      double a = ds_re[q], b = ds_im[q];
      block_sum2<BLK>(a, b);
      if (threadIdx.x == 0 && pok[q]) {
        const int gp = g0 + q;
        const int slot = gp / nz, z = gp - slot * nz;
        Partial P;
        if (DOT) {
          P.re = (double)scale * a; P.im = (double)scale * b; P.n2 = 0;
        } else {
          P.re = 0; P.im = 0; P.n2 = a / NN;  // |r|^2 of the updated residual
        }
        P.pad = 0;
        dpart[(long long)rhs_of(active, slot) * nz + z] = P;
      }
    }
  }
}

// Recursive z filter in mode space.  Thread (mode m, chunk c) owns planes
// [c L, c L + L) of one mode of one rhs, held in registers:
//   causal      F(z) = sum_k alpha_k F(z-k) + sum_k fb_k  r(z-k)
//   anti-causal B(z) = sum_k alpha_k B(z+k) + sum_k fbb_k r(z+1+k)
//   out(z) = F(z) + B(z),   alpha_k = -q_{nf-k}.
// Each chunk first runs both recursions from a zero state (the inputs of
// neighbouring planes are read as halo).  By linearity the missing part is
// the homogeneous response to the true state entering the chunk; those
// states follow from a short scan over the chunks with the state
// propagator M^L (M = companion matrix of the outgoing recurrence), and
// each thread then adds the homogeneous responses.  Block = 64 modes x C
// chunks (C <= 8) of one rhs.
template <typename T>
__device__ __forceinline__ void small_matvec(const cplx<T>* M, const cplx<T>* v, cplx<T>* out, int nf) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cplx<T> s = mk<T>(0, 0);
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (i < nf && j < nf) s = s + M[i * 3 + j] * v[j];
    out[i] = s;
  }
}

template <typename T>
__device__ __forceinline__ void small_matmul(const cplx<T>* A, const cplx<T>* B, cplx<T>* C, int nf) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<T> s = mk<T>(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (i < nf && j < nf && k < nf) s = s + A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}

// M^n for the state S = (F(z), F(z-1), ..., F(z-nf+1)): S(z+1) = M S(z).
template <typename T>
__device__ void state_power(const cplx<T>* al, int nf, int n, cplx<T>* P) {
  cplx<T> M[9], R[9], tmp[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) { M[i] = mk<T>(0, 0); R[i] = mk<T>(0, 0); }
#pragma unroll
  for (int j = 0; j < 3; ++j) M[j] = al[j];
  M[1 * 3 + 0] = mk<T>(1, 0);
  M[2 * 3 + 1] = mk<T>(1, 0);
  for (int i = 0; i < 3; ++i) R[i * 4] = mk<T>(1, 0);
  while (n > 0) {
    if (n & 1) {
      small_matmul(R, M, tmp, nf);
#pragma unroll
      for (int i = 0; i < 9; ++i) R[i] = tmp[i];
    }
    n >>= 1;
    if (n) {
      small_matmul(M, M, tmp, nf);
#pragma unroll
      for (int i = 0; i < 9; ++i) M[i] = tmp[i];
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) P[i] = R[i];
}

//
// With DOT (the preconditioner inside COCG), block b takes 32 modes k in
// lanes 0..31 and their partners -k in lanes 32..63 (zpair_mode), so that
// one wavefront holds both factors of the bilinear form in mode space
// (Parseval, with R = in and Z = out in natural FFT order)
//   sum_x r(x) z(x) = dscale * sum_k sum_z R(-k, z) Z(k, z),   dscale = 1 / Nxy,
// the partner's output coming from lane t ^ 32 (a mode that is its own
// partner uses its own).  The block's partial goes to dpart[rhs][b], and
// block 0 clears slots [nmb, nz) of its rhs, so that the nz slots per rhs
// read by the scalar step sum to the form.  This spares the inverse
// transform a read of R.
template <typename T, int L, int NF, bool DOT>
__global__ void __launch_bounds__(512) k_zfilter(int nz, int nmb, int nxy, const cplx<T>* __restrict__ in,
                                                  cplx<T>* __restrict__ out, const ModeData* __restrict__ modes,
                                                  const int* __restrict__ e_rhs, const int* __restrict__ active,
                                                  int nx, Partial* __restrict__ dpart, double dscale) {
  extern __shared__ char smem_raw[];
  const int C = blockDim.y;
  cplx<T>* sc = reinterpret_cast<cplx<T>*>(smem_raw);  // [C][64][3] causal end states
  cplx<T>* sb = sc + (size_t)C * 64 * 3;                // [C][64][3] anti-causal begin states
  const int slot = blockIdx.x / nmb;
  const int mb = blockIdx.x - slot * nmb;
  int m = mb * 64 + threadIdx.x;
  bool self = false;
  if constexpr (DOT) m = zpair_mode(mb * 32 + (threadIdx.x & 31), threadIdx.x >> 5, nxy / nx, nx, self);
  // one wavefront per chunk: the chunk index (and every plane offset below)
  // is wave-uniform, which keeps the load addresses in scalar registers
  const int c = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int rhs = rhs_of(active, slot);
  const long long base = (long long)rhs * nxy * nz;
  const bool live = m < nxy;
  const int z0 = c * L;
  constexpr int nf = NF;
  cplx<T> al[3], fb[3], fbb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) al[k] = fb[k] = fbb[k] = mk<T>(0, 0);
  if (live) {
    const ModeData& md = modes[(long long)e_rhs[rhs] * nxy + m];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      al[k] = -cvt<T>(md.q[nf - 1 - k]);
      fb[k] = cvt<T>(md.fb[k]);
      fbb[k] = cvt<T>(md.fbb[k]);
    }
  }
  // inputs of planes z0-2 .. z0+L+2
  cplx<T> rr[L + 5];
#pragma unroll
  for (int i = 0; i < L + 5; ++i) {
    const int z = z0 - 2 + i;
    rr[i] = (live && z >= 0 && z < nz) ? in[base + (long long)z * nxy + m] : mk<T>(0, 0);
  }
  cplx<T> y[L];
  // causal pass from a zero state
  cplx<T> h0 = mk<T>(0, 0), h1 = mk<T>(0, 0), h2 = mk<T>(0, 0);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    cplx<T> F = al[0] * h0 + fb[0] * rr[i + 2];
    if (NF > 1) F = F + al[1] * h1 + fb[1] * rr[i + 1];
    if (NF > 2) F = F + al[2] * h2 + fb[2] * rr[i];
    h2 = h1;
    h1 = h0;
    h0 = (z0 + i < nz) ? F : mk<T>(0, 0);
    y[i] = h0;
  }
  // chunk end state, (F(e), F(e-1), F(e-2)) at e = z0+L-1 (planes past nz are zero)
  const int sidx = (c * 64 + threadIdx.x) * 3;
  sc[sidx + 0] = h0;
  sc[sidx + 1] = h1;
  sc[sidx + 2] = h2;
  // anti-causal pass from a zero state
  h0 = h1 = h2 = mk<T>(0, 0);
#pragma unroll
  for (int i = L - 1; i >= 0; --i) {
    cplx<T> B = al[0] * h0 + fbb[0] * rr[i + 3];
    if (NF > 1) B = B + al[1] * h1 + fbb[1] * rr[i + 4];
    if (NF > 2) B = B + al[2] * h2 + fbb[2] * rr[i + 5];
    h2 = h1;
    h1 = h0;
    h0 = (z0 + i < nz) ? B : mk<T>(0, 0);
    y[i] = y[i] + h0;
  }
  sb[sidx + 0] = h0;  // (B(z0), B(z0+1), B(z0+2))
  sb[sidx + 1] = h1;
  sb[sidx + 2] = h2;
  __syncthreads();
  // scan over chunks: sc[c] <- true end state of chunk c, sb[c] <- true begin state
  if (c == 0 && live && C > 1) {
    cplx<T> ML[9], prev[3], tmp[3];
    state_power(al, nf, L, ML);
    prev[0] = prev[1] = prev[2] = mk<T>(0, 0);
    for (int cc = 0; cc < C - 1; ++cc) {
      cplx<T>* S = sc + (cc * 64 + threadIdx.x) * 3;
      small_matvec(ML, prev, tmp, nf);
      for (int k = 0; k < 3; ++k) prev[k] = S[k] + tmp[k];
      for (int k = 0; k < 3; ++k) S[k] = prev[k];
    }
    // anti-causal: the last chunk may be shorter
    const int Llast = nz - (C - 1) * L;
    cplx<T> Mlast[9];
    state_power(al, nf, Llast, Mlast);
    prev[0] = prev[1] = prev[2] = mk<T>(0, 0);
    for (int cc = C - 1; cc >= 1; --cc) {
      cplx<T>* S = sb + (cc * 64 + threadIdx.x) * 3;
      small_matvec(cc == C - 1 ? Mlast : ML, prev, tmp, nf);
      for (int k = 0; k < 3; ++k) prev[k] = S[k] + tmp[k];
      for (int k = 0; k < 3; ++k) S[k] = prev[k];
    }
  }
  __syncthreads();
  // (with DOT every lane stays for the exchange and the reduction below; a
  // lane without a mode carries zero coefficients and stores nothing)
  if (!DOT && !live) return;
  // homogeneous responses to the true incoming states
  if (c > 0) {
    const cplx<T>* S = sc + ((c - 1) * 64 + threadIdx.x) * 3;
    h0 = S[0];
    h1 = S[1];
    h2 = S[2];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      cplx<T> F = al[0] * h0;
      if (NF > 1) F = F + al[1] * h1;
      if (NF > 2) F = F + al[2] * h2;
      h2 = h1;
      h1 = h0;
      h0 = F;
      y[i] = y[i] + F;
    }
  }
  if (c < C - 1) {
    const cplx<T>* S = sb + ((c + 1) * 64 + threadIdx.x) * 3;
    h0 = S[0];
    h1 = S[1];
    h2 = S[2];
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
      cplx<T> B = al[0] * h0;
      if (NF > 1) B = B + al[1] * h1;
      if (NF > 2) B = B + al[2] * h2;
      h2 = h1;
      h1 = h0;
      h0 = B;
      y[i] = y[i] + B;
    }
  }
  if constexpr (DOT) {
    // the outputs are stored first, so that they drain while the partner
    // exchange and the block reduction run
    if (live) {
#pragma unroll
      for (int i = 0; i < L; ++i)
        if (z0 + i < nz) out[base + (long long)(z0 + i) * nxy + m] = y[i];
    }
    double a = 0, b = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      cplx<T> zp;
      zp.re = __shfl_xor(y[i].re, 32);
      zp.im = __shfl_xor(y[i].im, 32);
      if (self) zp = y[i];
      const cplx<T> rv = rr[i + 2];  // R(k, z0 + i); zero past nz and on lanes without a mode
      a += (double)rv.re * zp.re - (double)rv.im * zp.im;
      b += (double)rv.re * zp.im + (double)rv.im * zp.re;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o);
      b += __shfl_xor(b, o);
    }
    double* red = reinterpret_cast<double*>(sb + (size_t)C * 64 * 3);  // [C][2]
    if (threadIdx.x == 0) {
      red[2 * c] = a;
      red[2 * c + 1] = b;
    }
    __syncthreads();
    if (c == 0) {
      if (threadIdx.x == 0) {
        double sa = 0, sb2 = 0;
        for (int cc = 0; cc < C; ++cc) {
          sa += red[2 * cc];
          sb2 += red[2 * cc + 1];
        }
        Partial P;
        P.re = dscale * sa; P.im = dscale * sb2; P.n2 = 0; P.pad = 0;
        dpart[(long long)rhs * nz + mb] = P;
      }
      if (mb == 0) {
        Partial Z;
        Z.re = Z.im = Z.n2 = Z.pad = 0;
        for (int k = nmb + threadIdx.x; k < nz; k += 64) dpart[(long long)rhs * nz + k] = Z;
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < L; ++i)
    if (z0 + i < nz) out[base + (long long)(z0 + i) * nxy + m] = y[i];
}

// --------------------------------------------------------- right-hand side ---
// b on the nf planes facing the source electrode (Eq. (6)):
//   b(plane i from the source side, r) = btil_i * lat(r),
// lat = exp(i G.r) (kind 0), cos(G.r) (kind 1) or sin(G.r) (kind 2).
__device__ __forceinline__ double lateral_phase(int m, int nx, int ny, int p) {
  const int ix = m % nx, iy = m / nx;
  const int nux = ix < nx / 2 ? ix : ix - nx;
  const int nuy = iy < ny / 2 ? iy : iy - ny;
  const int j = p / nx, i = p - j * nx;
  // reduce the integer phase first for accuracy
  long long a = ((long long)nux * i) % nx;
  long long b = ((long long)nuy * j) % ny;
  return 2.0 * M_PI * ((double)a / nx + (double)b / ny);
}

// With faces_only the planes between the two faces are not written (the
// solver reads b on the 2 nf face planes only).
__global__ void k_rhs(int nx, int ny, int nz, int nf, const int* __restrict__ e_rhs,
                      const int* __restrict__ mode_rhs, const int* __restrict__ kind_rhs,
                      int side, const ModeData* __restrict__ modes, zd* __restrict__ b, int faces_only) {
  const int rhs = blockIdx.y;
  const int nxy = nx * ny;
  const long long vol = (long long)nxy * nz;
  const int m = mode_rhs[rhs];
  const int kind = kind_rhs[rhs];
  if (m < 0 || m >= nxy) return;  // ids are validated on the host
  const ModeData& md = modes[(long long)e_rhs[rhs] * nxy + m];
  const long long n = faces_only ? 2LL * nf * nxy : vol;
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n;
       j += (long long)gridDim.x * blockDim.x) {
    long long idx = j;
    if (faces_only && j >= (long long)nf * nxy) idx += (long long)(nz - 2 * nf) * nxy;  // the far face
    const int z = (int)(idx / nxy);
    const int p = (int)(idx - (long long)z * nxy);
    const int i = side ? nz - 1 - z : z;
    zd val = mk(0.0, 0.0);
    if (i < nf) {
      double ph = lateral_phase(m, nx, ny, p);
      double s, c;
      sincos(ph, &s, &c);
      zd lat = kind == 0 ? mk(c, s) : (kind == 1 ? mk(c, 0.0) : mk(s, 0.0));
      val = md.btil[i] * lat;
    }
    b[rhs * vol + idx] = val;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_dot(const cplx<T>* __restrict__ a, const cplx<T>* __restrict__ b,
                                             long long vol, int nblk, Partial* __restrict__ part,
                                             const int* __restrict__ active) {
  const int slot = blockIdx.x / nblk;
  const int blk = blockIdx.x - slot * nblk;
  const int rhs = rhs_of(active, slot);
  const cplx<T>* ar = a + rhs * vol;
  const cplx<T>* br = b + rhs * vol;
  const long long per = (vol + nblk - 1) / nblk;
  const long long i0 = blk * per, i1 = min(vol, i0 + per);
  double sre = 0, sim = 0, sn = 0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    cplx<T> u = ar[i], v = br[i];
    double ur = u.re, ui = u.im, vr = v.re, vi = v.im;
    sre += ur * vr - ui * vi;
    sim += ur * vi + ui * vr;
    sn += ur * ur + ui * ui;
  }
  block_reduce3(sre, sim, sn);
  if (threadIdx.x == 0) {
    Partial P;
    P.re = sre; P.im = sim; P.n2 = sn; P.pad = 0;
    part[(long long)rhs * nblk + blk] = P;
  }
}

// x += alpha p ; r -= alpha q ; partial |r|^2
// r -= alpha q with the partials of |r|^2 and r^T r (the solution update
// d += alpha p is applied by the next operator pass).
template <typename T>
__global__ void __launch_bounds__(256) k_update_r(cplx<T>* __restrict__ r, const cplx<T>* __restrict__ q,
                                                  const zd* __restrict__ alpha, long long vol, int nblk,
                                                  Partial* __restrict__ part, const int* __restrict__ active) {
  const int slot = blockIdx.x / nblk;
  const int blk = blockIdx.x - slot * nblk;
  const int rhs = rhs_of(active, slot);
  const cplx<T> a = cvt<T>(alpha[rhs]);
  const long long per = (vol + nblk - 1) / nblk;
  const long long i0 = blk * per, i1 = min(vol, i0 + per);
  const long long off = rhs * vol;
  double sn = 0, d0 = 0, d1 = 0;
  for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    cplx<T> rv = r[off + i] - a * q[off + i];
    r[off + i] = rv;
    sn += (double)rv.re * rv.re + (double)rv.im * rv.im;
    d0 += (double)rv.re * rv.re - (double)rv.im * rv.im;  // r^T r (for P = I)
    d1 += 2.0 * (double)rv.re * rv.im;
  }
  block_reduce3(sn, d0, d1);
  if (threadIdx.x == 0) {
    Partial P;
    P.re = d0; P.im = d1; P.n2 = sn; P.pad = 0;
    part[(long long)rhs * nblk + blk] = P;
  }
}

// Per-rhs scalars of COCG (device arrays indexed by rhs id).
struct Scal {
  zd* rho;
  zd* alpha;
  zd* beta;
  double* rn2;   // |r|^2 after the update
  int* flag;     // breakdown flags
  int* xset;     // FIN_NORM after a refinement: marks x as written (or nullptr)
  int* dlive;    // d holds data: set by FIN_ALPHA once the operator has applied a
                 // pending step (the old alpha was nonzero), cleared by FIN_NORM
                 // after a refinement has folded d into x (or nullptr)
};

// Scalar steps of the fused iteration, one wavefront per active rhs: the
// partials of each rhs are summed lane-strided and then across the lanes,
// a fixed order.
//   FIN_ALPHA    mu = sum pa (p^T A p); alpha = rho / mu (breakdown: alpha = 0, flag)
//   FIN_BETA     rho' = sum pa (r^T z); beta = rho' / rho; rho = rho';
//                rn2 = sum pb.n2 (|r|^2 written by the update)
//   FIN_RESTART  rho = sum pa (r^T z); beta = 0; flag cleared
//   FIN_NORM     rn2 = sum pa.n2
//   FIN_KEEP     after a residual replacement that keeps the direction:
//                rho' = sum pa (r^T z) of the replaced residual.  The last
//                FIN_BETA left beta = rho_{k+1} / rho_k and rho = rho_{k+1}
//                from the recursive residual; the direction update takes
//                the replaced one instead: beta = rho_k^-1 rho' =
//                beta rho' / rho; rho = rho'; alpha = 0 (the pending step is
//                already folded into x); flag cleared
enum { FIN_ALPHA = 0, FIN_BETA = 1, FIN_RESTART = 2, FIN_NORM = 3, FIN_KEEP = 4 };

__global__ void __launch_bounds__(256) k_finish2(Scal S, const Partial* __restrict__ pa, int na,
                                                 const Partial* __restrict__ pb, int nb, int mode,
                                                 const int* __restrict__ active, int nact) {
  const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (slot >= nact) return;  // whole wavefronts
  const int rhs = rhs_of(active, slot);
  double re = 0, im = 0, n2 = 0;
  for (int k = lane; k < na; k += 64) {
    const Partial P = pa[(long long)rhs * na + k];
    re += P.re;
    im += P.im;
    if (mode == FIN_NORM) n2 += P.n2;
  }
  if (pb)
    for (int k = lane; k < nb; k += 64) n2 += pb[(long long)rhs * nb + k].n2;
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off);
    im += __shfl_xor(im, off);
    n2 += __shfl_xor(n2, off);
  }
  if (lane != 0) return;
  if (mode == FIN_ALPHA) {
    const zd rho = S.rho[rhs];
    if (S.dlive && (S.alpha[rhs].re != 0 || S.alpha[rhs].im != 0)) S.dlive[rhs] = 1;
    const double d = re * re + im * im;
    if (!(d > 0) || !isfinite(d)) {
      S.alpha[rhs] = mk(0.0, 0.0);
      S.flag[rhs] = 1;
    } else {
      S.alpha[rhs] = mk((rho.re * re + rho.im * im) / d, (rho.im * re - rho.re * im) / d);
    }
  } else if (mode == FIN_BETA) {
    const zd rho = S.rho[rhs];
    const double d = rho.re * rho.re + rho.im * rho.im;
    if (!(d > 0) || !isfinite(re * re + im * im)) {
      S.beta[rhs] = mk(0.0, 0.0);
      S.flag[rhs] = 1;
    } else {
      S.beta[rhs] = mk((re * rho.re + im * rho.im) / d, (im * rho.re - re * rho.im) / d);
    }
    S.rho[rhs] = mk(re, im);
    S.rn2[rhs] = n2;
  } else if (mode == FIN_NORM) {
    S.rn2[rhs] = n2;
    if (S.xset) S.xset[rhs] = 1;
    if (S.dlive) S.dlive[rhs] = 0;
  } else if (mode == FIN_KEEP) {  // p_new = z + beta p_old next, no pending solution update
    const zd rho = S.rho[rhs];
    const double d = rho.re * rho.re + rho.im * rho.im;
    if (!(d > 0) || !isfinite(re * re + im * im)) {
      S.beta[rhs] = mk(0.0, 0.0);  // cannot continue the recurrence: restart instead
    } else {
      const zd q = mk((re * rho.re + im * rho.im) / d, (im * rho.re - re * rho.im) / d);  // rho' / rho
      S.beta[rhs] = S.beta[rhs] * q;
    }
    S.rho[rhs] = mk(re, im);
    S.alpha[rhs] = mk(0.0, 0.0);
    S.flag[rhs] = 0;
  } else {  // FIN_RESTART: p_new = z next, with no pending solution update
    S.rho[rhs] = mk(re, im);
    S.alpha[rhs] = mk(0.0, 0.0);
    S.beta[rhs] = mk(0.0, 0.0);
    S.flag[rhs] = 0;
  }
}

// y = b - y  (b nonzero only where the rhs kernel wrote it; stored in full)
template <typename T>
// y = b - y, with b read on the 2 nf face planes only (it vanishes between
// them)
__global__ void k_residual(const zd* __restrict__ b, cplx<T>* __restrict__ y, long long vol, long long lo,
                           long long hi, const int* __restrict__ active) {
  const int rhs = rhs_of(active, blockIdx.y);
  const long long off = rhs * vol;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x) {
    const zd bv = (i < lo || i >= hi) ? b[off + i] : mk(0.0, 0.0);
    cplx<T> yv = y[off + i];
    y[off + i] = mk<T>((T)bv.re - yv.re, (T)bv.im - yv.im);
  }
}

// dst (complex64) = src (complex128); dst zeroed when src == nullptr
template <typename TD, typename TS>
__global__ void k_convert(const cplx<TS>* __restrict__ src, cplx<TD>* __restrict__ dst, long long vol,
                          const int* __restrict__ active) {
  const int rhs = rhs_of(active, blockIdx.y);
  const long long off = rhs * vol;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x)
    dst[off + i] = src ? mk<TD>((TD)src[off + i].re, (TD)src[off + i].im) : mk<TD>(0, 0);
}

// x (complex128) += d + alpha p (complex64 or complex128).  x is not read
// where xset[rhs] = 0 (its first refinement), d not where dlive[rhs] = 0
// (no step applied since the last refinement); d is left as it is, and the
// refinement's norm step marks it dead.
template <typename T>
__global__ void k_accumulate(zd* __restrict__ x, const cplx<T>* __restrict__ d, const cplx<T>* __restrict__ p,
                             const zd* __restrict__ alpha, const int* __restrict__ xset,
                             const int* __restrict__ dlive, long long vol, const int* __restrict__ active) {
  const int rhs = rhs_of(active, blockIdx.y);
  const long long off = rhs * vol;
  const cplx<T> a = cvt<T>(alpha[rhs]);
  const bool pend = a.re != (T)0 || a.im != (T)0;
  const bool have_x = xset[rhs] != 0, have_d = dlive[rhs] != 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x) {
    const zd xv = have_x ? x[off + i] : mk(0.0, 0.0);
    cplx<T> dv = have_d ? d[off + i] : mk<T>(0, 0);
    if (pend) dv = dv + a * p[off + i];
    x[off + i] = mk(xv.re + (double)dv.re, xv.im + (double)dv.im);
  }
}

// ------------------------------------------------------------- readout ---
// Mode amplitudes at the two electrode faces (Eq. (7)): FFT of the nf planes
// facing each electrode, then for every open mode the propagating component
// of the outgoing expansion:  far side  a_far[nu] = sum_m lr_m psi~_nu(plane m from the far side),
//                             near side a_near[nu] = sum_m ll_m psi~_nu(plane m from the near side).
// Block (rhs, face); face 0 = near (source) side, 1 = far side.
__global__ void k_readout(FFTPlan2D plan, int nz, int nf, int side, const zd* __restrict__ x,
                          const ModeData* __restrict__ modes, const int* __restrict__ e_rhs,
                          const zd* __restrict__ twx, const zd* __restrict__ twy,
                          zd* __restrict__ amp_near, zd* __restrict__ amp_far) {
  extern __shared__ char smem_raw[];
  zd* buf = reinterpret_cast<zd*>(smem_raw);
  const int nxy = plan.x.n * plan.y.n;
  const int rhs = blockIdx.x >> 1;
  const int face = blockIdx.x & 1;
  const long long vol = (long long)nxy * nz;
  const ModeData* md = modes + (long long)e_rhs[rhs] * nxy;
  zd* P[4];
  for (int k = 0; k <= nf; ++k) P[k] = buf + k * nxy;
  // plane of index m (m = 0..nf-1) counted from the face: near face of a left
  // incidence is plane m, far face is plane nz-nf+m; mirrored for side 1.
  for (int k = 0; k < nf; ++k) {
    int plane;
    if (face == 1) plane = side == 0 ? nz - nf + k : nf - 1 - k;
    else plane = side == 0 ? k : nz - 1 - k;
    const zd* src = x + rhs * vol + (long long)plane * nxy;
    for (int p = threadIdx.x; p < nxy; p += blockDim.x) P[k][p] = src[p];
    __syncthreads();
    zd* res = fft2d_lds(P[k], P[nf], plan, twx, twy, -1);
    if (res != P[k]) { zd* t = P[k]; P[k] = P[nf]; P[nf] = t; }
  }
  const double inv = 1.0 / nxy;
  zd* out = (face == 1 ? amp_far : amp_near) + (long long)rhs * nxy;
  for (int m = threadIdx.x; m < nxy; m += blockDim.x) {
    zd a = mk(0.0, 0.0);
    if (md[m].flags & MODE_OPEN) {
      for (int k = 0; k < nf; ++k) a = a + (face == 1 ? md[m].lr[k] : md[m].ll[k]) * P[k][m];
      a = inv * a;
    }
    out[m] = a;
  }
}

// Combine real-lateral-basis solutions into plane-wave channels and form
// T and R (Landauer-Buttiker, Sec. III):  for request c with basis (ic, is, sgn):
//   t[nu] = a_far[ic][nu] + i sgn a_far[is][nu]   (is < 0: no sine part)
//   r[nu] = a_near[..] combined - delta_{nu,mu} kin_mu
//   T = sum_nu (v_nu / v_mu) |t|^2,  R likewise.
__global__ void k_combine(int nxy, const int* __restrict__ req_e, const int* __restrict__ req_mode,
                          const int* __restrict__ req_c, const int* __restrict__ req_s,
                          const int* __restrict__ req_sgn, const ModeData* __restrict__ modes,
                          const zd* __restrict__ amp_near, const zd* __restrict__ amp_far,
                          zd* __restrict__ t_out, zd* __restrict__ r_out, double* __restrict__ T,
                          double* __restrict__ R) {
  const int c = blockIdx.x;
  const int e = req_e[c], mu = req_mode[c];
  if (mu < 0 || mu >= nxy) return;  // ids are validated on the host
  const int ic = req_c[c], is = req_s[c];
  const double sg = (double)req_sgn[c];
  const ModeData* md = modes + (long long)e * nxy;
  const double vmu = md[mu].v;
  double sT = 0, sR = 0, d2 = 0;
  for (int nu = threadIdx.x; nu < nxy; nu += blockDim.x) {
    zd tf = amp_far[(long long)ic * nxy + nu];
    zd rn = amp_near[(long long)ic * nxy + nu];
    if (is >= 0) {
      zd tfs = amp_far[(long long)is * nxy + nu];
      zd rns = amp_near[(long long)is * nxy + nu];
      tf = tf + mk(-sg * tfs.im, sg * tfs.re);
      rn = rn + mk(-sg * rns.im, sg * rns.re);
    }
    if (nu == mu) rn = rn - md[mu].kin;
    t_out[(long long)c * nxy + nu] = tf;
    r_out[(long long)c * nxy + nu] = rn;
    if (md[nu].flags & MODE_OPEN) {
      sT += md[nu].v / vmu * norm2(tf);
      sR += md[nu].v / vmu * norm2(rn);
    }
  }
  block_reduce3(sT, sR, d2);
  if (threadIdx.x == 0) {
    T[c] = sT;
    R[c] = sR;
  }
}

// psi[c] = x[ic] + i sgn x[is]
template <typename TO>
__global__ void k_combine_psi(const zd* __restrict__ x, cplx<TO>* __restrict__ psi, long long vol,
                              const int* __restrict__ req_c, const int* __restrict__ req_s,
                              const int* __restrict__ req_sgn) {
  const int c = blockIdx.y;
  const int ic = req_c[c], is = req_s[c];
  const double sg = (double)req_sgn[c];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x) {
    zd v = x[(long long)ic * vol + i];
    if (is >= 0) {
      zd s = x[(long long)is * vol + i];
      v = v + mk(-sg * s.im, sg * s.re);
    }
    psi[(long long)c * vol + i] = mk<TO>((TO)v.re, (TO)v.im);
  }
}

}  // namespace

// =================================================================== host ===
int dot_blocks(iobm_ctx c);
StencilArgs stencil_args(iobm_ctx c, int zchunk) {
  StencilArgs S;
  S.nx = c->g.nx; S.ny = c->g.ny; S.nz = c->g.nz; S.nf = c->g.nf; S.nxy = c->g.nxy;
  S.zchunk = zchunk;
  S.nchunks = (c->g.nz + zchunk - 1) / zchunk;
  double ihx = 1.0 / (c->g.hx * c->g.hx), ihy = 1.0 / (c->g.hy * c->g.hy), ihz = 1.0 / (c->g.hz * c->g.hz);
  S.e0 = 0.5 * c->c[0] * (ihx + ihy + ihz);
  for (int n = 0; n < 4; ++n) {
    double cn = n <= c->g.nf ? c->c[n] : 0.0;
    S.wx[n] = 0.5 * cn * ihx;
    S.wy[n] = 0.5 * cn * ihy;
    S.wz[n] = 0.5 * cn * ihz;
  }
  return S;
}

template <typename T> static const cplx<T>* twx(iobm_ctx c);
template <> const zd* twx<double>(iobm_ctx c) { return c->twx_d; }
template <> const zf* twx<float>(iobm_ctx c) { return c->twx_f; }
template <typename T> static const cplx<T>* twy(iobm_ctx c);
template <> const zd* twy<double>(iobm_ctx c) { return c->twy_d; }
template <> const zf* twy<float>(iobm_ctx c) { return c->twy_f; }
template <typename T> static const cplx<T>* sigtab(iobm_ctx c);
template <> const zd* sigtab<double>(iobm_ctx c) { return c->sig_d; }
template <> const zf* sigtab<float>(iobm_ctx c) { return c->sig_f; }
template <typename T> static const T* Vptr(iobm_ctx c);
template <> const double* Vptr<double>(iobm_ctx c) { return c->V_d; }
template <> const float* Vptr<float>(iobm_ctx c) { return c->V_f; }

static int fft_threads(int nxy) {
  int t = 256;
  while (t < nxy && t < 1024) t *= 2;
  if (nxy < 256) t = ((nxy + 63) / 64) * 64;
  return t;
}

static int a25_max_threads(int ppt) {
  switch (ppt) {
    case 3: return A25<3>::max_threads;
    case 4: return A25<4>::max_threads;
    default: return A25<1>::max_threads;
  }
}

// Points-per-thread variants offered to the autotuner and to pinned shapes:
// 1..3, and 4 only for nf = 1 (with wider stencils its register window
// spills; 9 points per thread spilled at every order and is not built).
static bool a25_ppt_ok(iobm_ctx c, int ppt) {
  if (ppt < 1 || ppt > 4 || (ppt == 4 && c->g.nf > 1)) return false;
  const int threads = ((c->g.nxy + ppt - 1) / ppt + 63) / 64 * 64;
  return threads <= a25_max_threads(ppt);
}

// 2.5D stencil launch shape: points per thread (1, 2, 3 or 4; the block is
// ceil(nxy / ppt) threads rounded to a wavefront, at most the variant's
// bound) and planes per block.  Chosen by the autotuner below, pinned by
// the caller, else a default rule.
template <typename T, class Op>
static bool launch_apply25_shape(iobm_ctx c, int ppt, int zc, const Op& op, int nrhs, const double* E_rhs,
                                 const int* active) {
  const int nxy = c->g.nxy;
  if (!a25_ppt_ok(c, ppt)) return false;
  const int threads = ((nxy + ppt - 1) / ppt + 63) / 64 * 64;
  StencilArgs S = stencil_args(c, zc);
  if (S.nchunks > PQ_STENCIL_MAX) return false;
  size_t sh = 2 * (size_t)nxy * sizeof(cplx<T>);
  dim3 grid(nrhs * S.nchunks), blk(threads);
#define IOBM_A25(NF, MP) \
  hipLaunchKernelGGL((k_apply25<T, NF, MP, Op>), grid, blk, sh, c->stream, S, op, Vptr<T>(c), E_rhs, active)
#define IOBM_A25P(NF)                     \
  if (ppt == 1) { IOBM_A25(NF, 1); }      \
  else if (ppt == 2) { IOBM_A25(NF, 2); } \
  else { IOBM_A25(NF, 3); }
  switch (c->g.nf) {
    case 1:
      if (ppt == 4) { IOBM_A25(1, 4); }
      else { IOBM_A25P(1); }
      break;
    case 2: IOBM_A25P(2); break;
    default: IOBM_A25P(3); break;
  }
#undef IOBM_A25P
#undef IOBM_A25
  return true;
}

static int default_ppt(iobm_ctx c) {
  // the fewest points per thread that fit: the smallest register window
  for (int ppt : {1, 2, 3, 4})
    if (a25_ppt_ok(c, ppt)) return ppt;
  return 0;
}

// The stencil with any policy: the 2.5D kernel at the tuned (or default)
// shape, else the cache-based one.
template <typename T, class Op>
static hipError_t launch_stencil(iobm_ctx c, const Op& op, int nrhs, const double* E_rhs, const int* active,
                                 double bytes_per_point, int cls = 0) {
  const int rec = prof_start(c, cls ? cls : (sizeof(T) == 4 ? IOBM_K_STENCIL : IOBM_K_STENCIL_C128));
  bool done = false;
  const iobm_launch_shape& sh = c->shape[prec_index<T>()];
  if (sh.stencil != 2) {
    int ppt = sh.points_per_thread, zc = sh.planes_per_block;
    if (ppt <= 0) ppt = default_ppt(c);
    if (zc <= 0) zc = 32;
    // a small batch (the tail of a solve, a small refinement subset) gets
    // shorter chunks, so that there are blocks for every compute unit and no
    // block walks a long chunk alone
    while (zc > 8 && (long long)nrhs * ((c->g.nz + zc - 1) / zc) < 2LL * c->num_cu) zc /= 2;
    if (ppt > 0) done = launch_apply25_shape<T, Op>(c, ppt, zc, op, nrhs, E_rhs, active);
  }
  if (!done) {
    StencilArgs S = stencil_args(c, 16);
    if (S.nchunks > PQ_STENCIL_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_apply<T, Op>), dim3(nrhs * S.nchunks), dim3(256), 0, c->stream, S, op, Vptr<T>(c), E_rhs,
                       active);
  }
  prof_stop(c, rec, bytes_per_point * nrhs * c->g.npts);
  return hipGetLastError();
}

// The electrode term of the operator on the 2 nf face planes (see k_boundary).
// Algorithmic bytes: read x and y, write y (or the residual) on the faces.
template <typename T, typename TR, int N>
static void launch_boundary_reg(iobm_ctx c, const cplx<T>* x, cplx<T>* y, cplx<TR>* rout, int nrhs,
                                const int* e_rhs, const ModeData* modes, const int* active, Partial* part) {
#define IOBM_BREG(NF)                                                                                         \
  hipLaunchKernelGGL((k_boundary_reg<T, TR, N, NF>), dim3(2 * nrhs), dim3(N * NF), 0, c->stream, c->g.nz, x, y, \
                     rout, sigtab<T>(c), e_rhs, twx<T>(c), active, part, (int)PQ_SLOTS, (int)PQ_BOUNDARY)
  switch (c->g.nf) {
    case 1: IOBM_BREG(1); break;
    case 2: IOBM_BREG(2); break;
    default: IOBM_BREG(3); break;
  }
#undef IOBM_BREG
}

template <typename T, typename TR>
static hipError_t launch_boundary(iobm_ctx c, const cplx<T>* x, cplx<T>* y, cplx<TR>* rout, int nrhs,
                                  const int* e_rhs, const ModeData* modes, const int* active, Partial* part) {
  size_t sh = (size_t)(c->g.nf + 1) * c->g.nxy * sizeof(cplx<T>);
  const int rec = prof_start(c, IOBM_K_BOUNDARY);
  bool reg = c->g.nx == c->g.ny && c->shape[prec_index<T>()].plane_fft != 2;
  if (reg) {
    switch (c->g.nx) {
      case 8: launch_boundary_reg<T, TR, 8>(c, x, y, rout, nrhs, e_rhs, modes, active, part); break;
      case 12: launch_boundary_reg<T, TR, 12>(c, x, y, rout, nrhs, e_rhs, modes, active, part); break;
      case 16: launch_boundary_reg<T, TR, 16>(c, x, y, rout, nrhs, e_rhs, modes, active, part); break;
      case 24: launch_boundary_reg<T, TR, 24>(c, x, y, rout, nrhs, e_rhs, modes, active, part); break;
      case 32: launch_boundary_reg<T, TR, 32>(c, x, y, rout, nrhs, e_rhs, modes, active, part); break;
      case 48: launch_boundary_reg<T, TR, 48>(c, x, y, rout, nrhs, e_rhs, modes, active, part); break;
      default: reg = false;
    }
  }
  if (!reg)
    hipLaunchKernelGGL((k_boundary<T, TR>), dim3(2 * nrhs), dim3(fft_threads(c->g.nxy)), sh, c->stream, c->plan,
                       c->g.nz, c->g.nf, x, y, rout, sigtab<T>(c), e_rhs, twx<T>(c), twy<T>(c), active, part,
                       (int)PQ_SLOTS, (int)PQ_BOUNDARY);
  prof_stop(c, rec, (double)nrhs * 2 * c->g.nf * c->g.nxy * (2 * sizeof(cplx<T>) + sizeof(cplx<TR>)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bloch_stencil_fused(iobm_ctx c, const BlochPhase& ph, const BlochFuse<T>& F, cplx<T>* y, int nrhs,
                                      const double* E_rhs, const int* sgn, const int* active) {
  if (nrhs <= 0) return hipSuccess;
  const StencilArgs S = stencil_args(c, 16);
  OpBlochFuse<T> op;
  op.z = F.z;
  op.pold = F.pold;
  op.pnew = F.pnew;
  op.y = y;
  op.d = F.d;
  op.beta = F.beta;
  op.alpha = F.alpha;
  op.sgn = sgn;
  for (int n = 0; n < 4; ++n) {
    op.f[0][n] = cvt<T>(S.wx[n] * ph.x[n]);
    op.f[1][n] = cvt<T>(S.wy[n] * ph.y[n]);
  }
  // streams: read z, p_old, d; write p_new, y, d; the nfresh slots right
  // after a restart read z and write p_new and y only
  const int nf = std::min(std::max(F.nfresh, 0), nrhs);
  const double streams = 6.0 * (nrhs - nf) + 3.0 * nf;
  return launch_stencil<T, OpBlochFuse<T>>(c, op, nrhs, E_rhs, active, streams / nrhs * sizeof(cplx<T>),
                                            IOBM_K_BLOCH_STENCIL);
}
template hipError_t launch_bloch_stencil_fused<float>(iobm_ctx, const BlochPhase&, const BlochFuse<float>&, zf*, int,
                                                      const double*, const int*, const int*);
template hipError_t launch_bloch_stencil_fused<double>(iobm_ctx, const BlochPhase&, const BlochFuse<double>&, zd*,
                                                       int, const double*, const int*, const int*);

template <typename T>
hipError_t launch_face_sigma(iobm_ctx c, const cplx<T>* x, cplx<T>* y, int nrhs, const int* e_rhs,
                             const int* active) {
  if (nrhs <= 0) return hipSuccess;
  return launch_boundary<T, T>(c, x, y, nullptr, nrhs, e_rhs, c->modes_d, active, nullptr);
}
template hipError_t launch_face_sigma<float>(iobm_ctx, const zf*, zf*, int, const int*, const int*);
template hipError_t launch_face_sigma<double>(iobm_ctx, const zd*, zd*, int, const int*, const int*);

template <typename T>
hipError_t launch_apply(iobm_ctx c, const cplx<T>* x, cplx<T>* y, int nrhs, const double* E_rhs,
                        const int* e_rhs, const ModeData* modes, const int* active,
                        const ApplyFuse<T>* fuse) {
  if (nrhs <= 0) return hipSuccess;
  hipError_t err;
  Partial* part = nullptr;
  if (fuse) {
    OpFuseP<T> op{fuse->z, fuse->pold, fuse->beta, fuse->pnew, y, fuse->part, fuse->alpha, fuse->d, fuse->dlive};
    // streams: read z, p_old (and d); write p_new, y (and d); the nfresh
    // restarted rhs read z only, the nkept rhs right after a replacement
    // that kept the direction read z and p_old, the nfirst rhs after either
    // do not read d
    const int nf = std::min(std::max(fuse->nfresh, 0), nrhs);
    const int nk = std::min(std::max(fuse->nkept, 0), nrhs - nf);
    const int n1 = fuse->alpha ? std::min(std::max(fuse->nfirstd, 0), nrhs - nf - nk) : 0;
    const double full = fuse->alpha ? 6.0 : 4.0;
    err = launch_stencil<T>(c, op, nrhs, E_rhs, active,
                            (full * (nrhs - nf - nk - n1) + 5.0 * n1 + 4.0 * nk + 3.0 * nf) / nrhs *
                                sizeof(cplx<T>));
    x = fuse->pnew;  // the electrode and nonlocal terms read the assembled operand
    part = fuse->part;
  } else {
    OpPlain<T> op{x, y};
    err = launch_stencil<T>(c, op, nrhs, E_rhs, active, 2.0 * sizeof(cplx<T>));
  }
  if (err != hipSuccess) return err;
  err = launch_boundary<T, T>(c, x, y, nullptr, nrhs, e_rhs, modes, active, part);
  if (err != hipSuccess) return err;
  if (c->kb.ncen > 0) return launch_kb_apply<T>(c, x, y, nrhs, part, active);
  return hipSuccess;
}

template <typename TR>
hipError_t launch_refresh(iobm_ctx c, const zd* x, const zd* b, zd* rface, cplx<TR>* r, int nrhs,
                          const double* E_rhs, const int* e_rhs, const ModeData* modes, const int* active,
                          Partial* part) {
  if (nrhs <= 0) return hipSuccess;
  if (c->kb.ncen > 0) return hipErrorNotSupported;
  OpRefresh<TR> op{x, b, rface, r, part, c->g.nz, c->g.nf, c->g.nxy};
  hipError_t err = launch_stencil<double>(c, op, nrhs, E_rhs, active, (double)sizeof(zd) + sizeof(cplx<TR>));
  if (err != hipSuccess) return err;
  return launch_boundary<double, TR>(c, x, rface, r, nrhs, e_rhs, modes, active, part);
}

template hipError_t launch_refresh<float>(iobm_ctx, const zd*, const zd*, zd*, zf*, int, const double*, const int*,
                                          const ModeData*, const int*, Partial*);
template hipError_t launch_refresh<double>(iobm_ctx, const zd*, const zd*, zd*, zd*, int, const double*, const int*,
                                           const ModeData*, const int*, Partial*);

template <typename TR>
hipError_t launch_bloch_refresh(iobm_ctx c, const BlochPhase& ph, const zd* x, const zd* b, zd* rface, cplx<TR>* r,
                                int nrhs, const double* E_rhs, const int* e_rhs, const int* sgn, const int* active,
                                Partial* part) {
  if (nrhs <= 0) return hipSuccess;
  const StencilArgs S = stencil_args(c, 16);
  OpBlochRefresh<TR> op;
  op.x = x;
  op.b = b;
  op.rface = rface;
  op.r = r;
  op.part = part;
  op.nz = c->g.nz;
  op.nf = c->g.nf;
  op.nxy = c->g.nxy;
  op.sgn = sgn;
  for (int n = 0; n < 4; ++n) {
    op.f[0][n] = S.wx[n] * ph.x[n];
    op.f[1][n] = S.wy[n] * ph.y[n];
  }
  hipError_t err = launch_stencil<double>(c, op, nrhs, E_rhs, active, (double)sizeof(zd) + sizeof(cplx<TR>));
  if (err != hipSuccess) return err;
  return launch_boundary<double, TR>(c, x, rface, r, nrhs, e_rhs, c->modes_d, active, part);
}
template hipError_t launch_bloch_refresh<float>(iobm_ctx, const BlochPhase&, const zd*, const zd*, zd*, zf*, int,
                                                const double*, const int*, const int*, const int*, Partial*);
template hipError_t launch_bloch_refresh<double>(iobm_ctx, const BlochPhase&, const zd*, const zd*, zd*, zd*, int,
                                                 const double*, const int*, const int*, const int*, Partial*);

template <typename T>
hipError_t launch_precond_laplacian(iobm_ctx c, double alpha, const cplx<T>* r, cplx<T>* z, int nrhs,
                                    const int* active, Partial* dpart) {
  if (nrhs <= 0) return hipSuccess;
  StencilArgs S = stencil_args(c, 16);
  const int rec = prof_start(c, IOBM_K_PRECOND_LAP);
  hipLaunchKernelGGL(k_precond_lap<T>, dim3(nrhs * S.nchunks), dim3(256), 0, c->stream, S,
                     (T)exp(-alpha), r, z, active, dpart);
  prof_stop(c, rec, 2.0 * nrhs * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_precond_jacobi(iobm_ctx c, const cplx<T>* r, cplx<T>* z, int nrhs, const int* e_rhs,
                                 const double* E_rhs, const int* active, Partial* dpart) {
  if (nrhs <= 0) return hipSuccess;
  const int nblk = dot_blocks(c);
  const StencilArgs S = stencil_args(c, 16);
  const int rec = prof_start(c, IOBM_K_PRECOND_JACOBI);
  hipLaunchKernelGGL(k_precond_jacobi<T>, dim3(nrhs * nblk), dim3(256), 0, c->stream, r, z, c->V_d, c->kb.diag_d,
                     c->sdiag_d, e_rhs, E_rhs, S.e0, c->g.nz, c->g.nf, c->g.nxy, nblk, active, dpart);
  prof_stop(c, rec, 2.0 * nrhs * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}
template hipError_t launch_precond_jacobi<float>(iobm_ctx, const zf*, zf*, int, const int*, const double*, const int*,
                                                 Partial*);
template hipError_t launch_precond_jacobi<double>(iobm_ctx, const zd*, zd*, int, const int*, const double*,
                                                  const int*, Partial*);

hipError_t launch_sigma_diag(iobm_ctx c, int nE) {
  if (nE <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sigma_diag, dim3(nE * c->g.nf), dim3(256), 0, c->stream, c->sig_d, c->g.nxy, c->g.nf,
                     c->sdiag_d);
  return hipGetLastError();
}

template <typename T, int N, int PPB>
static void launch_fft_reg(iobm_ctx c, const cplx<T>* in, cplx<T>* out, int sign, double scale, int nrhs,
                           const int* active, const cplx<T>* mvec, Partial* dpart, const FftUpd<T>* upd) {
  const int nplanes = nrhs * c->g.nz;
  const dim3 grid((nplanes + PPB - 1) / PPB), blk(fft_split<T, N>() * N * PPB);
  const FftUpd<T> U = upd ? *upd : FftUpd<T>();
  if (upd)
    hipLaunchKernelGGL((k_fft_planes_reg<T, N, PPB, FFT_UPDATE>), grid, blk, 0, c->stream, c->g.nz, nplanes, in, out,
                       twx<T>(c), sign, (T)scale, active, mvec, dpart, U);
  else if (dpart)
    hipLaunchKernelGGL((k_fft_planes_reg<T, N, PPB, FFT_DOT>), grid, blk, 0, c->stream, c->g.nz, nplanes, in, out,
                       twx<T>(c), sign, (T)scale, active, mvec, dpart, U);
  else
    hipLaunchKernelGGL((k_fft_planes_reg<T, N, PPB, FFT_PLAIN>), grid, blk, 0, c->stream, c->g.nz, nplanes, in, out,
                       twx<T>(c), sign, (T)scale, active, mvec, dpart, U);
}

static bool square_reg_size(iobm_ctx c) {
  if (c->g.nx != c->g.ny) return false;
  switch (c->g.nx) {
    case 8: case 12: case 16: case 24: case 32: case 48: return true;
    default: return false;
  }
}

// planes per block of the register FFT (measured: one plane per block is
// fastest at 48 x 48)
template <typename T>
bool fft_reg_available(iobm_ctx c) {
  return square_reg_size(c) && c->shape[prec_index<T>()].plane_fft != 2;
}
template bool fft_reg_available<float>(iobm_ctx);
template bool fft_reg_available<double>(iobm_ctx);

template <typename T>
static bool fft_reg_dispatch(iobm_ctx c, const cplx<T>* in, cplx<T>* out, int sign, double scale, int nrhs,
                             const int* active, const cplx<T>* mvec, Partial* dpart, const FftUpd<T>* upd) {
  if (!fft_reg_available<T>(c)) return false;
  switch (c->g.nx) {
    case 8: launch_fft_reg<T, 8, 16>(c, in, out, sign, scale, nrhs, active, mvec, dpart, upd); return true;
    case 12: launch_fft_reg<T, 12, 8>(c, in, out, sign, scale, nrhs, active, mvec, dpart, upd); return true;
    case 16: launch_fft_reg<T, 16, 8>(c, in, out, sign, scale, nrhs, active, mvec, dpart, upd); return true;
    case 24: launch_fft_reg<T, 24, 4>(c, in, out, sign, scale, nrhs, active, mvec, dpart, upd); return true;
    case 32: launch_fft_reg<T, 32, 4>(c, in, out, sign, scale, nrhs, active, mvec, dpart, upd); return true;
    default: launch_fft_reg<T, 48, 1>(c, in, out, sign, scale, nrhs, active, mvec, dpart, upd); return true;
  }
}

// Batched plane FFTs; with dpart set, also the per-plane partials of
// out^T r (dpart[rhs][z]): from r itself (dvec) in the LDS kernel, by
// Parseval from mvec = the forward FFT of r in the register kernel.
template <typename T>
hipError_t launch_fft_planes(iobm_ctx c, const cplx<T>* in, cplx<T>* out, int sign, double scale, int nrhs,
                             const int* active, const cplx<T>* dvec = nullptr, const cplx<T>* mvec = nullptr,
                             Partial* dpart = nullptr, const FftUpd<T>* upd = nullptr) {
  if (nrhs <= 0) return hipSuccess;
  if (upd && !fft_reg_available<T>(c)) return hipErrorInvalidValue;
  const int rec = prof_start(c, upd ? IOBM_K_FFT_PLANES_UPD : (dpart ? IOBM_K_FFT_PLANES_DOT : IOBM_K_FFT_PLANES));
  if (!fft_reg_dispatch<T>(c, in, out, sign, scale, nrhs, active, mvec, dpart, upd)) {
    size_t sh = 2 * (size_t)c->g.nxy * sizeof(cplx<T>);
    hipLaunchKernelGGL(k_fft_planes<T>, dim3(nrhs * c->g.nz), dim3(256), sh, c->stream, c->plan, c->g.nz, in, out,
                       twx<T>(c), twy<T>(c), sign, (T)scale, active, dvec, dpart);
  }
  // streams: plain 2; with the dot 3 (read Z, R; write z); with the update 3
  // (read q, R; write R)
  prof_stop(c, rec, (upd ? 3.0 : (dpart ? 3.0 : 2.0)) * nrhs * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

// chunk length of the z filter (tuned per context and precision)
// With dpart (requires zfilter_dot_ok), the paired layout and the partials of
// the bilinear form r^T z, dpart[rhs][0..nz).
template <typename T>
static hipError_t launch_zfilter(iobm_ctx c, int L, const cplx<T>* in, cplx<T>* out, int nrhs, const int* e_rhs,
                                 const ModeData* modes, const int* active, Partial* dpart = nullptr) {
  const int nxy = c->g.nxy, nz = c->g.nz;
  const bool dot = dpart != nullptr;
  const int nmb = dot ? c->zpair_nmb : (nxy + 63) / 64;
  const int C = (nz + L - 1) / L;
  size_t sh = 2 * (size_t)C * 64 * 3 * sizeof(cplx<T>) + (dot ? 2 * (size_t)C * sizeof(double) : 0);
  const double dscale = 1.0 / nxy;
  const int rec = prof_start(c, IOBM_K_ZFILTER);
#define IOBM_ZF3(LL, NFF, DD)                                                                                     \
  hipLaunchKernelGGL((k_zfilter<T, LL, NFF, DD>), dim3(nrhs * nmb), dim3(64, C), sh, c->stream, nz, nmb, nxy, in, \
                     out, modes, e_rhs, active, c->g.nx, dpart, dscale)
#define IOBM_ZF2(LL, NFF)        \
  if (dot) IOBM_ZF3(LL, NFF, true); \
  else IOBM_ZF3(LL, NFF, false)
#define IOBM_ZF(LL)                                   \
  switch (c->g.nf) {                                  \
    case 1: IOBM_ZF2(LL, 1); break;                   \
    case 2: IOBM_ZF2(LL, 2); break;                   \
    default: IOBM_ZF2(LL, 3); break;                  \
  }
  switch (L) {
    case 8: IOBM_ZF(8); break;
    case 16: IOBM_ZF(16); break;
    default: IOBM_ZF(32); break;
  }
#undef IOBM_ZF
#undef IOBM_ZF2
#undef IOBM_ZF3
  prof_stop(c, rec, 2.0 * nrhs * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

// The z filter takes the r^T z partials when the plane transforms are the
// register ones (natural mode order, R in the scratch that feeds the filter),
// its pair blocks fit the nz partial slots of a rhs, and the launch shape
// does not name the inverse transform (rz_pass 2).
static bool zfilter_dot_fits(iobm_ctx c) { return c->zpair_nmb > 0 && c->zpair_nmb <= c->g.nz; }
template <typename T>
static bool zfilter_dot_ok(iobm_ctx c) {
  return zfilter_dot_fits(c) && fft_reg_available<T>(c) && c->shape[prec_index<T>()].rz_pass != 2;
}

static int default_zfilter_chunk(iobm_ctx c) {
  // at most 8 chunks (512 threads per block)
  int L = 16;
  if ((c->g.nz + L - 1) / L > 8) L = 32;
  return L;
}

template <typename T>
static int zfilter_chunk(iobm_ctx c) {
  const int tuned = c->shape[prec_index<T>()].zfilter_chunk;
  return tuned > 0 ? tuned : default_zfilter_chunk(c);
}

template <typename T>
hipError_t launch_precond_fft(iobm_ctx c, const cplx<T>* r, cplx<T>* z, cplx<T>* scratch, int nrhs,
                              const int* e_rhs, const ModeData* modes, const int* active, Partial* dpart,
                              const FftUpd<T>* upd) {
  if (nrhs <= 0) return hipSuccess;
  const int L = zfilter_chunk<T>(c);
  if ((c->g.nz + L - 1) / L > 8) return hipErrorInvalidValue;
  const int rec = prof_start(c, IOBM_K_PRECOND_FFT);
  // with upd, scratch holds the residual in mode space and is updated from q
  hipError_t err = launch_fft_planes<T>(c, upd ? upd->q : r, scratch, -1, 1.0, nrhs, active, nullptr, nullptr,
                                        upd ? upd->n2part : nullptr, upd);
  const bool zdot = dpart != nullptr && zfilter_dot_ok<T>(c);
  if (err == hipSuccess) err = launch_zfilter<T>(c, L, scratch, z, nrhs, e_rhs, modes, active, zdot ? dpart : nullptr);
  if (err == hipSuccess && zdot) err = launch_fft_planes<T>(c, z, z, +1, 1.0 / c->g.nxy, nrhs, active);
  else if (err == hipSuccess)
    err = launch_fft_planes<T>(c, z, z, +1, 1.0 / c->g.nxy, nrhs, active, r, scratch, dpart);
  prof_stop(c, rec, 2.0 * nrhs * c->g.npts * sizeof(cplx<T>));
  return err;
}

// Autotuner: time every admissible (points per thread, planes per block)
// shape of the 2.5D stencil and every z-filter chunk length once on the
// caller's own batch (x -> y, y is scratch), keep the fastest per precision.
// With rz_part (nrhs x nz partials), the z filter is timed as the
// preconditioner will run it: with the r^T z partials where it takes them.
template <typename T>
void autotune(iobm_ctx c, const cplx<T>* x, cplx<T>* y, cplx<T>* scratch, int nrhs, const double* E_rhs,
              const int* e_rhs, const ModeData* modes, const int* active, const ApplyFuse<T>* fuse,
              Partial* rz_part) {
  bool& done = c->tuned[prec_index<T>()];
  if (done || nrhs <= 0) return;
  done = true;
  iobm_launch_shape& sh = c->shape[prec_index<T>()];
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return;
  if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
  auto timed = [&](auto&& fn) -> float {
    fn();  // warm-up (first launch of a shape)
    (void)hipEventRecord(a, c->stream);
    fn();
    fn();
    (void)hipEventRecord(b, c->stream);
    float ms = 1e30f;
    if (hipEventSynchronize(b) == hipSuccess && hipGetLastError() == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  };
  if (sh.stencil != 2) {
    // the shape is timed on the operator as the iteration runs it
    float best = 1e30f;
    int bp = 0, bz = 0;
    for (int ppt : {1, 2, 3, 4})
      for (int zc : {16, 32, 64}) {
        if (!a25_ppt_ok(c, ppt)) continue;
        if (zc > c->g.nz && zc != 16) continue;
        float t = timed([&] {
          if (fuse)
            launch_apply25_shape<T>(c, ppt, zc,
                                    OpFuseP<T>{fuse->z, fuse->pold, fuse->beta, fuse->pnew, y, fuse->part,
                                               fuse->alpha, fuse->d, fuse->dlive},
                                    nrhs, E_rhs, active);
          else
            launch_apply25_shape<T>(c, ppt, zc, OpPlain<T>{x, y}, nrhs, E_rhs, active);
        });
        if (t < best) { best = t; bp = ppt; bz = zc; }
      }
    if (bp > 0) { sh.stencil = 1; sh.points_per_thread = bp; sh.planes_per_block = bz; }
  }
  if (scratch) {
    // the z filter's chunk length and, where the z filter can take the r^T z
    // partials, which pass takes them: each composition is timed with the
    // inverse transform that follows the filter (plain after the filter's
    // dot, with the dot from R otherwise)
    const bool try_dot = rz_part != nullptr && zfilter_dot_ok<T>(c);
    float best = 1e30f;
    int bl = 0, bd = 0;
    for (int dot = 0; dot <= (try_dot ? 1 : 0); ++dot)
      for (int L : {8, 16, 32}) {
        if ((c->g.nz + L - 1) / L > 8) continue;
        float t = timed([&] {
          (void)launch_zfilter<T>(c, L, scratch, y, nrhs, e_rhs, modes, active, dot ? rz_part : nullptr);
          if (try_dot && dot)
            (void)launch_fft_planes<T>(c, y, y, +1, 1.0 / c->g.nxy, nrhs, active);
          else if (try_dot)
            (void)launch_fft_planes<T>(c, y, y, +1, 1.0 / c->g.nxy, nrhs, active, nullptr, scratch, rz_part);
        });
        if (t < best) { best = t; bl = L; bd = dot; }
      }
    if (bl > 0) sh.zfilter_chunk = bl;
    if (try_dot && bl > 0) sh.rz_pass = bd ? 1 : 2;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}

template void autotune<float>(iobm_ctx, const zf*, zf*, zf*, int, const double*, const int*, const ModeData*,
                              const int*, const ApplyFuse<float>*, Partial*);
template void autotune<double>(iobm_ctx, const zd*, zd*, zd*, int, const double*, const int*, const ModeData*,
                               const int*, const ApplyFuse<double>*, Partial*);

template hipError_t launch_apply<double>(iobm_ctx, const zd*, zd*, int, const double*, const int*,
                                         const ModeData*, const int*, const ApplyFuse<double>*);
template hipError_t launch_apply<float>(iobm_ctx, const zf*, zf*, int, const double*, const int*,
                                        const ModeData*, const int*, const ApplyFuse<float>*);
template hipError_t launch_precond_laplacian<double>(iobm_ctx, double, const zd*, zd*, int, const int*, Partial*);
template hipError_t launch_precond_laplacian<float>(iobm_ctx, double, const zf*, zf*, int, const int*, Partial*);
template hipError_t launch_precond_fft<double>(iobm_ctx, const zd*, zd*, zd*, int, const int*,
                                               const ModeData*, const int*, Partial*, const FftUpd<double>*);
template hipError_t launch_precond_fft<float>(iobm_ctx, const zf*, zf*, zf*, int, const int*,
                                              const ModeData*, const int*, Partial*, const FftUpd<float>*);

bool launch_shape_valid(iobm_ctx c, int prec, const iobm_launch_shape& s, std::string& why) {
  (void)prec;
  if (s.stencil < 0 || s.stencil > 2 || s.plane_fft < 0 || s.plane_fft > 2) {
    why = "stencil and plane_fft must be 0, 1 or 2";
    return false;
  }
  if (s.points_per_thread != 0 && !a25_ppt_ok(c, s.points_per_thread)) {
    why = "points_per_thread does not fit this plane size / FD order";
    return false;
  }
  if (s.stencil == 1 && s.points_per_thread == 0 && default_ppt(c) == 0) {
    why = "no 2.5D stencil variant fits this plane size";
    return false;
  }
  const int zc = s.planes_per_block;
  if (zc != 0 && zc != 8 && zc != 16 && zc != 32 && zc != 64) {
    why = "planes_per_block must be 8, 16, 32 or 64";
    return false;
  }
  const int L = s.zfilter_chunk;
  if (L != 0 && ((L != 8 && L != 16 && L != 32) || (c->g.nz + L - 1) / L > 8)) {
    why = "zfilter_chunk must be 8, 16 or 32 with at most 8 chunks along z";
    return false;
  }
  if (s.plane_fft == 1 && !square_reg_size(c)) {
    why = "the in-register plane FFT needs square planes of 8, 12, 16, 24, 32 or 48 points";
    return false;
  }
  return true;
}

iobm_launch_shape launch_shape_in_effect(iobm_ctx c, int prec) {
  const iobm_launch_shape& s = c->shape[prec];
  iobm_launch_shape r;
  const int ppt = s.points_per_thread > 0 ? s.points_per_thread : default_ppt(c);
  r.stencil = (s.stencil == 2 || ppt == 0) ? 2 : 1;
  r.points_per_thread = r.stencil == 1 ? ppt : 0;
  r.planes_per_block = r.stencil == 1 ? (s.planes_per_block > 0 ? s.planes_per_block : 32) : 16;
  r.zfilter_chunk = s.zfilter_chunk > 0 ? s.zfilter_chunk : default_zfilter_chunk(c);
  r.plane_fft = (square_reg_size(c) && s.plane_fft != 2) ? 1 : 2;
  r.rz_pass = (r.plane_fft == 1 && zfilter_dot_fits(c) && s.rz_pass != 2) ? 1 : 2;
  return r;
}

// partials of r^T z per rhs written by each preconditioner (P = I: the
// update kernel's r^T r, one per reduction block)
int dot_blocks(iobm_ctx c);
int precond_slots(iobm_ctx c, int precond) {
  if (precond == IOBM_PC_LATERAL_FFT) return c->g.nz;
  if (precond == IOBM_PC_JACOBI) return dot_blocks(c);
  if (precond == IOBM_PC_TRUNCATED_LAPLACIAN) return (c->g.nz + 15) / 16;
  return dot_blocks(c);
}

// ---- small launchers used by the solver ------------------------------------
static dim3 vol_grid(long long vol, int nrhs) {
  long long b = (vol + 255) / 256;
  if (b > 1024) b = 1024;
  return dim3((unsigned)b, (unsigned)nrhs);
}

hipError_t launch_rhs(iobm_ctx c, int nrhs, const int* e_rhs, const int* mode_rhs, const int* kind_rhs,
                      int side, const ModeData* modes, zd* b, bool faces_only) {
  if (nrhs <= 0) return hipSuccess;
  const bool fo = faces_only && c->g.nz >= 2 * c->g.nf;
  const long long n = fo ? 2LL * c->g.nf * c->g.nxy : c->g.npts;
  hipLaunchKernelGGL(k_rhs, vol_grid(n, nrhs), dim3(256), 0, c->stream, c->g.nx, c->g.ny, c->g.nz, c->g.nf,
                     e_rhs, mode_rhs, kind_rhs, side, modes, b, fo ? 1 : 0);
  return hipGetLastError();
}

// |b|^2 per rhs over the 2 nf face planes (b vanishes between them), one
// partial per rhs
__global__ void __launch_bounds__(256) k_face_norm2(const zd* __restrict__ b, long long vol, int nxy, int nz, int nf,
                                                    Partial* __restrict__ part, const int* __restrict__ active) {
  const int rhs = rhs_of(active, blockIdx.x);
  const zd* br = b + rhs * vol;
  const long long n = 2LL * nf * nxy, far = (long long)(nz - 2 * nf) * nxy;
  double s = 0, d0 = 0, d1 = 0;
  for (long long j = threadIdx.x; j < n; j += blockDim.x) {
    const zd v = br[j < (long long)nf * nxy ? j : j + far];
    s += v.re * v.re + v.im * v.im;
  }
  block_reduce3(s, d0, d1);
  if (threadIdx.x == 0) {
    Partial P;
    P.re = P.im = P.pad = 0;
    P.n2 = s;
    part[rhs] = P;
  }
}

hipError_t launch_face_norm2(iobm_ctx c, const zd* b, int nact, const int* active, Partial* part) {
  if (nact <= 0) return hipSuccess;
  if (c->g.nz < 2 * c->g.nf) return hipErrorInvalidValue;
  const int rec = prof_start(c, IOBM_K_DOT);
  hipLaunchKernelGGL(k_face_norm2, dim3(nact), dim3(256), 0, c->stream, b, c->g.npts, c->g.nxy, c->g.nz, c->g.nf,
                     part, active);
  prof_stop(c, rec, (double)nact * 2 * c->g.nf * c->g.nxy * sizeof(zd));
  return hipGetLastError();
}

// The start of an iteration from x = 0: r = b (b read on the face planes
// only).
template <typename T>
__global__ void __launch_bounds__(256) k_init_r(const zd* __restrict__ b, cplx<T>* __restrict__ r, long long vol,
                                                int nxy, int nz, int nf, const int* __restrict__ active) {
  const int rhs = rhs_of(active, blockIdx.y);
  const long long off = rhs * vol, lo = (long long)nf * nxy, hi = (long long)(nz - nf) * nxy;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < vol;
       i += (long long)gridDim.x * blockDim.x) {
    cplx<T> v = mk<T>(0, 0);
    if (i < lo || i >= hi) v = mk<T>((T)b[off + i].re, (T)b[off + i].im);
    r[off + i] = v;
  }
}

template <typename T>
hipError_t launch_init_r(iobm_ctx c, const zd* b, cplx<T>* r, int nact, const int* active) {
  if (nact <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_r<T>, vol_grid(c->g.npts, nact), dim3(256), 0, c->stream, b, r, c->g.npts, c->g.nxy,
                     c->g.nz, c->g.nf, active);
  return hipGetLastError();
}
template hipError_t launch_init_r<float>(iobm_ctx, const zd*, zf*, int, const int*);
template hipError_t launch_init_r<double>(iobm_ctx, const zd*, zd*, int, const int*);

int dot_blocks(iobm_ctx c) {
  long long vol = c->g.npts;
  long long b = vol / 8192;
  if (b < 1) b = 1;
  if (b > 64) b = 64;
  return (int)b;
}

template <typename T>
hipError_t launch_dot(iobm_ctx c, const cplx<T>* a, const cplx<T>* b, int nact, const int* active,
                      void* part) {
  if (nact <= 0) return hipSuccess;
  int nblk = dot_blocks(c);
  const int rec = prof_start(c, IOBM_K_DOT);
  hipLaunchKernelGGL(k_dot<T>, dim3(nact * nblk), dim3(256), 0, c->stream, a, b, c->g.npts, nblk,
                     (Partial*)part, active);
  prof_stop(c, rec, (a == b ? 1.0 : 2.0) * nact * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update_r(iobm_ctx c, cplx<T>* r, const cplx<T>* q, const zd* alpha, int nact, const int* active,
                           void* part) {
  if (nact <= 0) return hipSuccess;
  int nblk = dot_blocks(c);
  const int rec = prof_start(c, IOBM_K_UPDATE);
  hipLaunchKernelGGL(k_update_r<T>, dim3(nact * nblk), dim3(256), 0, c->stream, r, q, alpha, c->g.npts, nblk,
                     (Partial*)part, active);
  prof_stop(c, rec, 3.0 * nact * c->g.npts * sizeof(cplx<T>));
  return hipGetLastError();
}

hipError_t launch_finish2(iobm_ctx c, zd* rho, zd* alpha, zd* beta, double* rn2, int* flag, const Partial* pa,
                          int na, const Partial* pb, int nb, int mode, int nact, const int* active, int* xset,
                          int* dlive) {
  if (nact <= 0) return hipSuccess;
  Scal S;
  S.rho = rho; S.alpha = alpha; S.beta = beta; S.rn2 = rn2; S.flag = flag; S.xset = xset; S.dlive = dlive;
  hipLaunchKernelGGL(k_finish2, dim3((nact + 3) / 4), dim3(256), 0, c->stream, S, pa, na, pb, nb, mode, active,
                     nact);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(iobm_ctx c, const zd* b, cplx<T>* y, int nact, const int* active) {
  if (nact <= 0) return hipSuccess;
  const long long lo = (long long)c->g.nf * c->g.nxy, hi = (long long)(c->g.nz - c->g.nf) * c->g.nxy;
  hipLaunchKernelGGL(k_residual<T>, vol_grid(c->g.npts, nact), dim3(256), 0, c->stream, b, y, c->g.npts, lo, hi,
                     active);
  return hipGetLastError();
}

template <typename TD, typename TS>
hipError_t launch_convert(iobm_ctx c, const cplx<TS>* src, cplx<TD>* dst, int nact, const int* active) {
  if (nact <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_convert<TD, TS>), vol_grid(c->g.npts, nact), dim3(256), 0, c->stream, src, dst,
                     c->g.npts, active);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_accumulate(iobm_ctx c, zd* x, const cplx<T>* d, const cplx<T>* p, const zd* alpha,
                             const int* xset, const int* dlive, int nact, const int* active, int nfirst, int ndead) {
  if (nact <= 0) return hipSuccess;
  const int rec = prof_start(c, IOBM_K_ACCUMULATE);
  hipLaunchKernelGGL(k_accumulate<T>, vol_grid(c->g.npts, nact), dim3(256), 0, c->stream, x, d, p, alpha, xset,
                     dlive, c->g.npts, active);
  // read x (not at the first refinement of the nfirst rhs), d (not for the
  // ndead rhs), p; write x
  prof_stop(c, rec, c->g.npts * ((double)nact * (sizeof(zd) + sizeof(cplx<T>)) + (double)(nact - nfirst) * sizeof(zd) +
                                 (double)(nact - ndead) * sizeof(cplx<T>)));
  return hipGetLastError();
}

hipError_t launch_readout(iobm_ctx c, int nrhs, int side, const zd* x, const ModeData* modes,
                          const int* e_rhs, zd* amp_near, zd* amp_far) {
  if (nrhs <= 0) return hipSuccess;
  size_t sh = (size_t)(c->g.nf + 1) * c->g.nxy * sizeof(zd);
  hipLaunchKernelGGL(k_readout, dim3(2 * nrhs), dim3(fft_threads(c->g.nxy)), sh, c->stream, c->plan, c->g.nz,
                     c->g.nf, side, x, modes, e_rhs, c->twx_d, c->twy_d, amp_near, amp_far);
  return hipGetLastError();
}

hipError_t launch_combine(iobm_ctx c, int nreq, const int* req_e, const int* req_mode, const int* req_c,
                          const int* req_s, const int* req_sgn, const ModeData* modes, const zd* amp_near,
                          const zd* amp_far, zd* t_out, zd* r_out, double* T, double* R) {
  if (nreq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3(nreq), dim3(256), 0, c->stream, c->g.nxy, req_e, req_mode, req_c, req_s,
                     req_sgn, modes, amp_near, amp_far, t_out, r_out, T, R);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_combine_psi(iobm_ctx c, int nreq, const zd* x, cplx<TO>* psi, const int* req_c,
                              const int* req_s, const int* req_sgn) {
  if (nreq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine_psi<TO>, vol_grid(c->g.npts, nreq), dim3(256), 0, c->stream, x, psi,
                     c->g.npts, req_c, req_s, req_sgn);
  return hipGetLastError();
}

template hipError_t launch_dot<double>(iobm_ctx, const zd*, const zd*, int, const int*, void*);
template hipError_t launch_dot<float>(iobm_ctx, const zf*, const zf*, int, const int*, void*);
template hipError_t launch_update_r<double>(iobm_ctx, zd*, const zd*, const zd*, int,
                                                     const int*, void*);
template hipError_t launch_update_r<float>(iobm_ctx, zf*, const zf*, const zd*, int,
                                                   const int*, void*);
template hipError_t launch_residual<double>(iobm_ctx, const zd*, zd*, int, const int*);
template hipError_t launch_residual<float>(iobm_ctx, const zd*, zf*, int, const int*);
template hipError_t launch_convert<float, double>(iobm_ctx, const zd*, zf*, int, const int*);
template hipError_t launch_convert<double, double>(iobm_ctx, const zd*, zd*, int, const int*);
template hipError_t launch_convert<float, float>(iobm_ctx, const zf*, zf*, int, const int*);
template hipError_t launch_accumulate<float>(iobm_ctx, zd*, const zf*, const zf*, const zd*, const int*,
                                            const int*, int, const int*, int, int);
template hipError_t launch_accumulate<double>(iobm_ctx, zd*, const zd*, const zd*, const zd*, const int*,
                                             const int*, int, const int*, int, int);
template hipError_t launch_combine_psi<double>(iobm_ctx, int, const zd*, zd*, const int*, const int*,
                                               const int*);
template hipError_t launch_combine_psi<float>(iobm_ctx, int, const zd*, zf*, const int*, const int*,
                                              const int*);
