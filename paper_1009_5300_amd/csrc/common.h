// Shared device/host definitions of libiobm: complex arithmetic, grid
// description, the lateral FFT plan and the LDS Stockham FFT used by the
// self-energy application, the lateral-Fourier preconditioner and readout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define IOBM_HD __host__ __device__ __forceinline__

template <typename T>
struct cplx {
  T re, im;
};

template <typename T> IOBM_HD cplx<T> mk(T r, T i) { cplx<T> c; c.re = r; c.im = i; return c; }
template <typename T> IOBM_HD cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> IOBM_HD cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> IOBM_HD cplx<T> operator-(cplx<T> a) { return mk(-a.re, -a.im); }
template <typename T> IOBM_HD cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> IOBM_HD cplx<T> operator*(T s, cplx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T> IOBM_HD cplx<T> conj(cplx<T> a) { return mk(a.re, -a.im); }
template <typename T> IOBM_HD T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// a + b*c
template <typename T> IOBM_HD cplx<T> cfma(cplx<T> b, cplx<T> c, cplx<T> a) {
  return mk(a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re);
}
template <typename T, typename U> IOBM_HD cplx<T> cvt(cplx<U> a) { return mk<T>((T)a.re, (T)a.im); }

typedef cplx<double> zd;
typedef cplx<float> zf;

// ---------------------------------------------------------------- grid ----
struct GridDev {
  int nx, ny, nz, nf;
  int nxy;
  long long npts;
  double hx, hy, hz;
};

// --------------------------------------------------------- FFT plan -------
// Mixed-radix factorisation of one lateral length (radices 4, 2, then odd
// primes), consumed by the Stockham stages below.
#define IOBM_FFT_MAXSTAGES 12
struct FFTPlan1D {
  int n;
  int nstages;
  int radix[IOBM_FFT_MAXSTAGES];
};

struct FFTPlan2D {
  FFTPlan1D x, y;
};

// In-LDS 2D FFT of one nx*ny plane (row-major, x fastest).  `tw` tables hold
// exp(-2 pi i k / n) for the forward transform; sign = -1 forward, +1
// inverse (unnormalised).  All threads of the block take part; the caller
// synchronises before (data written to `a`) and the function ends with a
// barrier.  Returns the buffer that holds the result (a or b).
template <typename T>
__device__ __forceinline__ cplx<T> twid(const cplx<T>* tw, int k, int sign) {
  cplx<T> w = tw[k];
  return sign < 0 ? w : conj(w);
}

// Radix-R butterfly on v[0..R-1]: v'[s] = sum_r v[r] exp(sign 2 pi i r s / R).
template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T>* v, const cplx<T>* tw, int n, int sign) {
  if constexpr (R == 2) {
    cplx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    cplx<T> a = v[0], b = v[1], c = v[2], d = v[3];
    cplx<T> s0 = a + c, s1 = a - c, s2 = b + d, s3 = b - d;
    // forward multiplies s3 by -i, inverse by +i
    cplx<T> js3 = sign < 0 ? mk(s3.im, -s3.re) : mk(-s3.im, s3.re);
    v[0] = s0 + s2;
    v[1] = s1 + js3;
    v[2] = s0 - s2;
    v[3] = s1 - js3;
  } else {
    cplx<T> in[R];
#pragma unroll
    for (int r = 0; r < R; ++r) in[r] = v[r];
    const int stride = n / R;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      cplx<T> acc = in[0];
#pragma unroll
      for (int r = 1; r < R; ++r) acc = cfma(in[r], twid(tw, ((r * s) % R) * stride, sign), acc);
      v[s] = acc;
    }
  }
}

// One Stockham pass of radix R over `count` independent 1D transforms of
// length n; element e of transform t lives at t*tstride + e*estride.  Ns is
// the length of the sub-transforms already completed by earlier passes.
template <typename T, int R>
__device__ void stockham_pass_r(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, int n,
                                int Ns, int count, int estride, int tstride, const cplx<T>* tw,
                                int sign) {
  const int per = n / R;
  const int total = count * per;
  const int tstep = n / (Ns * R);
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int t = w / per;
    const int j = w - t * per;
    const int base = t * tstride;
    const int k = j % Ns;
    cplx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx<T> a = in[base + (j + r * per) * estride];
      if (r && k) a = a * twid(tw, (r * k * tstep) % n, sign);
      v[r] = a;
    }
    dft_small<T, R>(v, tw, n, sign);
    const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + (idxD + r * Ns) * estride] = v[r];
  }
}

// Generic odd-prime radix (up to 31): O(R^2) butterfly, slow path for
// lateral sizes with unusual prime factors.
template <typename T>
__device__ void stockham_pass_generic(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                      int n, int R, int Ns, int count, int estride, int tstride,
                                      const cplx<T>* tw, int sign) {
  const int per = n / R;
  const int total = count * per;
  const int tstep = n / (Ns * R);
  const int stride = n / R;
  for (int w = threadIdx.x; w < total; w += blockDim.x) {
    const int t = w / per;
    const int j = w - t * per;
    const int base = t * tstride;
    const int k = j % Ns;
    const int idxD = (j / Ns) * Ns * R + k;
    for (int s = 0; s < R; ++s) {
      cplx<T> acc = mk<T>(0, 0);
      for (int r = 0; r < R; ++r) {
        cplx<T> a = in[base + (j + r * per) * estride];
        if (r && k) a = a * twid(tw, (r * k * tstep) % n, sign);
        acc = cfma(a, twid(tw, ((r * s) % R) * stride, sign), acc);
      }
      out[base + (idxD + s * Ns) * estride] = acc;
    }
  }
}

template <typename T>
__device__ __forceinline__ void stockham_pass(const cplx<T>* __restrict__ in,
                                              cplx<T>* __restrict__ out, int n, int R, int Ns,
                                              int count, int estride, int tstride,
                                              const cplx<T>* tw, int sign) {
  switch (R) {
    case 2: stockham_pass_r<T, 2>(in, out, n, Ns, count, estride, tstride, tw, sign); break;
    case 3: stockham_pass_r<T, 3>(in, out, n, Ns, count, estride, tstride, tw, sign); break;
    case 4: stockham_pass_r<T, 4>(in, out, n, Ns, count, estride, tstride, tw, sign); break;
    case 5: stockham_pass_r<T, 5>(in, out, n, Ns, count, estride, tstride, tw, sign); break;
    default: stockham_pass_generic(in, out, n, R, Ns, count, estride, tstride, tw, sign); break;
  }
}

template <typename T>
__device__ cplx<T>* fft2d_lds(cplx<T>* a, cplx<T>* b, const FFTPlan2D& p, const cplx<T>* twx,
                              const cplx<T>* twy, int sign) {
  const int nx = p.x.n, ny = p.y.n;
  cplx<T>* src = a;
  cplx<T>* dst = b;
  int Ns = 1;
  for (int s = 0; s < p.x.nstages; ++s) {  // rows: ny transforms, contiguous
    stockham_pass(src, dst, nx, p.x.radix[s], Ns, ny, 1, nx, twx, sign);
    Ns *= p.x.radix[s];
    __syncthreads();
    cplx<T>* t = src; src = dst; dst = t;
  }
  Ns = 1;
  for (int s = 0; s < p.y.nstages; ++s) {  // columns: nx transforms, stride nx
    stockham_pass(src, dst, ny, p.y.radix[s], Ns, nx, nx, 1, twy, sign);
    Ns *= p.y.radix[s];
    __syncthreads();
    cplx<T>* t = src; src = dst; dst = t;
  }
  return src;
}

// ------------------------------------------------ in-register 1D FFT ------
// Length-N transform held in registers (N known at compile time), same
// Stockham stages as above with every index a compile-time constant.
constexpr int pick_radix(int m) {
  return m % 4 == 0 ? 4 : (m % 2 == 0 ? 2 : (m % 3 == 0 ? 3 : (m % 5 == 0 ? 5 : m)));
}
constexpr int count_stages(int n) {
  int c = 0;
  for (int m = n; m > 1; m /= pick_radix(m)) ++c;
  return c;
}

template <typename T, int N, int Ns>
__device__ __forceinline__ void reg_fft_stages(cplx<T>* a, cplx<T>* b, const cplx<T>* tw, int sign) {
  if constexpr (Ns < N) {
    constexpr int R = pick_radix(N / Ns);
    constexpr int per = N / R;
    constexpr int tstep = N / (Ns * R);
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int k = j % Ns;
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cplx<T> x = a[j + r * per];
        if (r && k) x = x * twid(tw, (r * k * tstep) % N, sign);
        v[r] = x;
      }
      dft_small<T, R>(v, tw, N, sign);
      const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) b[idxD + r * Ns] = v[r];
    }
    reg_fft_stages<T, N, Ns * R>(b, a, tw, sign);
  }
}

// x <- DFT_N(x), sign -1 forward / +1 inverse (unnormalised); tw[k] = exp(-2 pi i k / N)
template <typename T, int N>
__device__ __forceinline__ void reg_fft(cplx<T>* x, const cplx<T>* tw, int sign) {
  cplx<T> y[N];
  reg_fft_stages<T, N, 1>(x, y, tw, sign);
  if constexpr (count_stages(N) % 2 == 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = y[i];
  }
}
