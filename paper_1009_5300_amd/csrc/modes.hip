// Electrode mode setup (FP64): for every energy and lateral mode of the
// periodic cross-section, the outgoing generalized Bloch states of the
// semi-infinite jellium lead and everything derived from them.
//
// Lead recurrence in one lateral mode (Eq. (2) generalised to nf planes):
//     sum_{n=-nf}^{nf} a_|n| psi(k+n) = (E - eps_nu) psi(k),  a_n = -chat_n / (2 hz^2),
// with eps_nu the lateral kinetic energy of the mode (Eq. (13) for nf = 1).
// With x = exp(i kz hz) and c = (x + 1/x)/2 the characteristic equation is a
// polynomial of degree nf in c (Chebyshev form); each c root gives a pair
// x, 1/x.  The outgoing (retarded) state of each pair is the decaying one,
// or, on the unit circle, the one with positive group velocity, which for
// the monotone 2nd/4th/6th-order dispersion is Im x > 0 (the branch rule
// after Eq. (13)).
//
// From the nf outgoing roots x_j:
//   q      monic polynomial prod_j (x - x_j);  its companion matrix M maps the
//          values of an outgoing combination on nf consecutive planes one
//          plane further, so the lead values beyond the boundary planes are
//          M^nf times the boundary values;
//   sig    right self-energy Sigma_R = W M^nf, W = couplings of the last nf
//          planes to the first nf lead planes; this is Eq. (10) with
//          Q^tra(lead) Q^tra(boundary)^-1 = M^nf, written without the
//          Vandermonde inverse (robust when two evanescent roots nearly meet);
//          for nf = 1 it is Eq. (15), -exp(i kz hz)/(2 hz^2);
//   fb,fbb flat-wire Green's function G(d) = <z+d|(E - H_0 - Sigma)^-1|z> of the
//          mode (the inverse used by the lateral-Fourier preconditioner), as an
//          order-nf recursive filter: G(d >= 0) obeys the outgoing recurrence,
//          G(0..nf-1) solve the nf central rows of the infinite-lead equation;
//   lr,ll  rows selecting the propagating component of the outgoing /
//          reflected expansion on nf boundary planes (Eq. (7)), as Lagrange
//          basis coefficients;
//   btil   incident right-hand side profile on planes 0..nf-1 (Eq. (6)):
//          couplings to Phi_in on the lead planes minus Sigma_L Phi_in.
#include <math.h>

#include "internal.h"

namespace {

IOBM_HD zd csqrt_(zd z) {
  double r = sqrt(z.re * z.re + z.im * z.im);
  double a = sqrt(fmax(0.0, 0.5 * (r + z.re)));
  double b = sqrt(fmax(0.0, 0.5 * (r - z.re)));
  if (z.im < 0) b = -b;
  return mk(a, b);
}
IOBM_HD zd cdiv(zd a, zd b) {
  double d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
IOBM_HD double cabs_(zd a) { return sqrt(a.re * a.re + a.im * a.im); }
IOBM_HD zd cpow_(zd x, int n) {
  zd r = mk(1.0, 0.0);
  if (n >= 0) {
    for (int i = 0; i < n; ++i) r = r * x;
  } else {
    zd y = cdiv(mk(1.0, 0.0), x);
    for (int i = 0; i < -n; ++i) r = r * y;
  }
  return r;
}

// Real roots and complex pairs of a*c^2 + b*c + d (a != 0), stable form.
IOBM_HD void quad_roots(double a, double b, double d, zd* r) {
  double disc = b * b - 4 * a * d;
  if (disc >= 0) {
    double s = sqrt(disc);
    double qq = -0.5 * (b + (b >= 0 ? s : -s));
    if (qq == 0) {
      r[0] = mk(0.0, 0.0);
      r[1] = mk(0.0, 0.0);
    } else {
      r[0] = mk(qq / a, 0.0);
      r[1] = mk(d / qq, 0.0);
    }
  } else {
    double s = sqrt(-disc);
    r[0] = mk(-b / (2 * a), s / (2 * a));
    r[1] = mk(-b / (2 * a), -s / (2 * a));
  }
}

// Roots of the monic cubic c^3 + p2 c^2 + p1 c + p0 with real coefficients:
// one real root by bracketed bisection + Newton, the rest from the deflated
// quadratic.
IOBM_HD void cubic_roots(double p2, double p1, double p0, zd* r) {
  double B = 1.0 + fmax(fabs(p2), fmax(fabs(p1), fabs(p0)));
  double lo = -B, hi = B;
  
  double flo = ((lo + p2) * lo + p1) * lo + p0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    double fm = ((mid + p2) * mid + p1) * mid + p0;
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
    if (hi - lo <= 1e-16 * fmax(1.0, fabs(mid))) break;
  }
  double c0 = 0.5 * (lo + hi);
  for (int it = 0; it < 3; ++it) {
    double fv = ((c0 + p2) * c0 + p1) * c0 + p0, df = (3 * c0 + 2 * p2) * c0 + p1;
    if (df != 0) c0 -= fv / df;
  }
  // deflate: c^2 + (p2 + c0) c + (p1 + c0 (p2 + c0))
  double b1 = p2 + c0, b0 = p1 + c0 * b1;
  quad_roots(1.0, b1, b0, r + 1);
  r[0] = mk(c0, 0.0);
}

// Newton polish of a (possibly complex) root of the Chebyshev-form
// polynomial P(c) = sum_k pc[k] c^k.
IOBM_HD zd polish(const double* pc, int deg, zd c) {
  for (int it = 0; it < 3; ++it) {
    zd f = mk(pc[deg], 0.0), df = mk(0.0, 0.0);
    for (int k = deg - 1; k >= 0; --k) {
      df = df * c + f;
      f = f * c + mk(pc[k], 0.0);
    }
    if (df.re == 0 && df.im == 0) break;
    zd st = cdiv(f, df);
    c = c - st;
  }
  return c;
}

// Small complex Gaussian elimination with partial pivoting, n <= 3.
IOBM_HD bool csolve(zd* A, zd* b, int n) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = cabs_(A[k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = cabs_(A[i * n + k]);
      if (v > best) { best = v; p = i; }
    }
    if (best == 0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) { zd t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
      zd t = b[k]; b[k] = b[p]; b[p] = t;
    }
    for (int i = k + 1; i < n; ++i) {
      zd f = cdiv(A[i * n + k], A[k * n + k]);
      for (int j = k; j < n; ++j) A[i * n + j] = A[i * n + j] - f * A[k * n + j];
      b[i] = b[i] - f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    zd s = b[k];
    for (int j = k + 1; j < n; ++j) s = s - A[k * n + j] * b[j];
    b[k] = cdiv(s, A[k * n + k]);
  }
  return true;
}

// Coefficients (ascending, monic implied) of prod_{j != skip} (x - r_j) over n nodes.
IOBM_HD void poly_from_roots(const zd* r, int n, int skip, zd* coef, int* deg) {
  zd p[4] = {mk(1.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  int d = 0;
  for (int j = 0; j < n; ++j) {
    if (j == skip) continue;
    // p(x) *= (x - r_j)
    for (int k = d + 1; k >= 1; --k) p[k] = p[k - 1] - r[j] * p[k];
    p[0] = -(r[j] * p[0]);
    ++d;
  }
  for (int k = 0; k <= d; ++k) coef[k] = p[k];
  *deg = d;
}

// Lagrange row: coefficients L_m (m < n) of the basis polynomial that is 1 at
// node r[p] and 0 at the other nodes.
IOBM_HD void lagrange_row(const zd* r, int n, int p, zd* L) {
  zd coef[4];
  int deg;
  poly_from_roots(r, n, p, coef, &deg);
  zd den = mk(1.0, 0.0);
  for (int j = 0; j < n; ++j)
    if (j != p) den = den * (r[p] - r[j]);
  for (int m = 0; m < n; ++m) L[m] = m <= deg ? cdiv(coef[m], den) : mk(0.0, 0.0);
}

}  // namespace

__host__ __device__ void compute_mode(const ModeArgs& A, double E, int m, ModeData* out) {
  const int nf = A.nf;
  const double* c = A.c;
  ModeData md;
  for (int i = 0; i < 9; ++i) md.sig[i] = mk(0.0, 0.0);
  for (int i = 0; i < 3; ++i) {
    md.q[i] = md.fb[i] = md.fbb[i] = md.lr[i] = md.ll[i] = md.btil[i] = mk(0.0, 0.0);
  }
  md.xp = md.kin = mk(0.0, 0.0);
  md.v = 0;
  md.flags = 0;
  md.pad_ = 0;

  // lateral kinetic energy of the plane wave (FFT-order mode numbers)
  const int ix = m % A.nx, iy = m / A.nx;
  const int nux = ix < A.nx / 2 ? ix : ix - A.nx;
  const int nuy = iy < A.ny / 2 ? iy : iy - A.ny;
  // (G_nu + kappa) h per direction
  const double thx = 2.0 * M_PI * nux / A.nx + A.tx, thy = 2.0 * M_PI * nuy / A.ny + A.ty;
  double ex = c[0], ey = c[0];
  for (int n = 1; n <= nf; ++n) {
    ex += 2.0 * c[n] * cos(n * thx);
    ey += 2.0 * c[n] * cos(n * thy);
  }
  const double eps = -ex / (2.0 * A.hx * A.hx) - ey / (2.0 * A.hy * A.hy);
  md.eps = eps;
  const double dE = E - eps;
  const double hz2 = A.hz * A.hz;

  // Chebyshev-form characteristic polynomial in c:
  //   chat_0 + 2 sum_n chat_n T_n(c) + 2 hz^2 dE = 0
  double pc[4] = {c[0] + 2.0 * hz2 * dE, 0, 0, 0};
  if (nf >= 1) pc[1] += 2.0 * c[1];
  if (nf >= 2) { pc[2] += 4.0 * c[2]; pc[0] -= 2.0 * c[2]; }
  if (nf >= 3) { pc[3] += 8.0 * c[3]; pc[1] -= 6.0 * c[3]; }
  zd croot[3];
  if (nf == 1) {
    croot[0] = mk(-pc[0] / pc[1], 0.0);
  } else if (nf == 2) {
    quad_roots(pc[2], pc[1], pc[0], croot);
  } else {
    cubic_roots(pc[2] / pc[3], pc[1] / pc[3], pc[0] / pc[3], croot);
  }
  for (int j = 0; j < nf; ++j) croot[j] = polish(pc, nf, croot[j]);

  // outgoing root of each pair
  zd x[3];
  int prop = -1;
  for (int j = 0; j < nf; ++j) {
    zd cc = croot[j];
    bool real = fabs(cc.im) <= 1e-14 * fmax(1.0, fabs(cc.re));
    if (real && fabs(fabs(cc.re) - 1.0) < 1e-9) md.flags |= MODE_THRESHOLD;
    if (real && fabs(cc.re) < 1.0) {
      x[j] = mk(cc.re, sqrt(1.0 - cc.re * cc.re));
      if (prop >= 0) md.flags |= MODE_FAIL;
      prop = j;
    } else {
      if (real) cc.im = 0.0;
      zd s = csqrt_(cc * cc - mk(1.0, 0.0));
      zd x1 = cc - s, x2 = cc + s;
      x[j] = cabs_(x1) < cabs_(x2) ? x1 : x2;
    }
  }
  // distinct outgoing roots are required by the Lagrange readout of the
  // propagating component only
  // monic outgoing polynomial
  {
    zd coef[4];
    int deg;
    poly_from_roots(x, nf, -1, coef, &deg);
    for (int k = 0; k < nf; ++k) md.q[k] = coef[k];
  }
  // companion matrix M (state = values on nf consecutive planes)
  zd Mc[9], Mp[9], tmp[9];
  for (int i = 0; i < nf * nf; ++i) Mc[i] = mk(0.0, 0.0);
  for (int i = 0; i + 1 < nf; ++i) Mc[i * nf + i + 1] = mk(1.0, 0.0);
  for (int k = 0; k < nf; ++k) Mc[(nf - 1) * nf + k] = -md.q[k];
  // Mp = M^nf
  for (int i = 0; i < nf * nf; ++i) Mp[i] = mk((i % (nf + 1)) == 0 ? 1.0 : 0.0, 0.0);
  for (int p = 0; p < nf; ++p) {
    for (int i = 0; i < nf; ++i)
      for (int j = 0; j < nf; ++j) {
        zd s = mk(0.0, 0.0);
        for (int k = 0; k < nf; ++k) s = s + Mp[i * nf + k] * Mc[k * nf + j];
        tmp[i * nf + j] = s;
      }
    for (int i = 0; i < nf * nf; ++i) Mp[i] = tmp[i];
  }
  double a[4];
  for (int n = 0; n <= nf; ++n) a[n] = -c[n] / (2.0 * hz2);
  // Sigma_R = W M^nf, W[i][m] = a_{nf+m-i} for m <= i
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < nf; ++j) {
      zd s = mk(0.0, 0.0);
      for (int mm = 0; mm <= i; ++mm) s = s + a[nf + mm - i] * Mp[mm * nf + j];
      md.sig[i * nf + j] = s;
    }

  // flat-wire Green's function: u_k^T = e_0^T M^k, k = 0..2nf
  zd U[7][3];
  for (int j = 0; j < nf; ++j) U[0][j] = mk(j == 0 ? 1.0 : 0.0, 0.0);
  for (int k = 1; k <= 2 * nf; ++k)
    for (int j = 0; j < nf; ++j) {
      zd s = mk(0.0, 0.0);
      for (int l = 0; l < nf; ++l) s = s + U[k - 1][l] * Mc[l * nf + j];
      U[k][j] = s;
    }
  // rows d = 0..nf-1: sum_n A_n G(|d - n|) = delta_d0, A_0 = dE - a_0, A_n = -a_|n|
  zd K[9], g[3];
  for (int d = 0; d < nf; ++d) {
    for (int j = 0; j < nf; ++j) K[d * nf + j] = mk(0.0, 0.0);
    for (int n = -nf; n <= nf; ++n) {
      double An = n == 0 ? dE - a[0] : -a[n < 0 ? -n : n];
      int dist = d - n < 0 ? n - d : d - n;
      for (int j = 0; j < nf; ++j) K[d * nf + j] = K[d * nf + j] + An * U[dist][j];
    }
    g[d] = mk(d == 0 ? 1.0 : 0.0, 0.0);
  }
  if (!csolve(K, g, nf)) md.flags |= MODE_FAIL;
  zd G[4];
  for (int d = 0; d <= nf; ++d) {
    zd s = mk(0.0, 0.0);
    for (int j = 0; j < nf; ++j) s = s + U[d][j] * g[j];
    G[d] = s;
  }
  for (int d = 0; d < nf; ++d) {
    zd s0 = G[d], s1 = G[d + 1];
    for (int k = 1; k <= d; ++k) {
      s0 = s0 + md.q[nf - k] * G[d - k];
      s1 = s1 + md.q[nf - k] * G[d + 1 - k];
    }
    md.fb[d] = s0;
    md.fbb[d] = s1;
  }

  if (prop >= 0) {
    md.flags |= MODE_OPEN;
    zd xp = x[prop];
    md.xp = xp;
    double v = 0;
    for (int n = 1; n <= nf; ++n) v += n * c[n] * cpow_(xp, n).im;
    md.v = v / A.hz;
    if (!(md.v > 0)) md.flags |= MODE_FAIL;
    lagrange_row(x, nf, prop, md.lr);
    zd y[3];
    for (int j = 0; j < nf; ++j) y[j] = cdiv(mk(1.0, 0.0), x[j]);
    lagrange_row(y, nf, prop, md.ll);
    zd kin = mk(0.0, 0.0);
    for (int mm = 0; mm < nf; ++mm) kin = kin + md.ll[mm] * cpow_(xp, mm);
    md.kin = kin;
    // right-hand side profile, planes i = 0..nf-1:
    //   sum_{m>=1, i+m<=nf} a_{i+m} xp^{-m} - sum_j SigmaL[i][j] xp^j,
    //   SigmaL[i][j] = SigmaR[nf-1-i][nf-1-j]
    for (int i = 0; i < nf; ++i) {
      zd s = mk(0.0, 0.0);
      for (int mm = 1; i + mm <= nf; ++mm) s = s + a[i + mm] * cpow_(xp, -mm);
      for (int j = 0; j < nf; ++j) s = s - md.sig[(nf - 1 - i) * nf + (nf - 1 - j)] * cpow_(xp, j);
      md.btil[i] = s;
    }
  }
  *out = md;
}

namespace {
__global__ void k_modes(ModeArgs A, const double* __restrict__ Elist, const double* __restrict__ kap,
                        ModeData* __restrict__ out) {
  const int nxy = A.nx * A.ny;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)nxy * A.nE) return;
  const int e = (int)(gid / nxy);
  const int m = (int)(gid - (long long)e * nxy);
  if (kap) {
    A.tx = kap[2 * e];
    A.ty = kap[2 * e + 1];
  }
  compute_mode(A, Elist[e], m, &out[gid]);
}
}  // namespace

hipError_t launch_modes(iobm_ctx ctx, const double* E_d, int nE, ModeData* out, const double* kap_d) {
  ModeArgs A;
  A.nx = ctx->g.nx;
  A.ny = ctx->g.ny;
  A.nf = ctx->g.nf;
  A.nE = nE;
  A.hx = ctx->g.hx;
  A.hy = ctx->g.hy;
  A.hz = ctx->g.hz;
  for (int i = 0; i < 4; ++i) A.c[i] = ctx->c[i];
  long long n = (long long)ctx->g.nxy * nE;
  int threads = 128;
  long long blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(k_modes, dim3((unsigned)blocks), dim3(threads), 0, ctx->stream, A, E_d, kap_d, out);
  return hipGetLastError();
}

namespace {
// Sigma_R blocks copied out of the mode table into [energy][nf * nf][mode]
// order, in complex128 and complex64, and the mode flags into [energy][mode].
__global__ void k_sigma_tables(int nE, int nxy, int nf, const ModeData* __restrict__ modes, zd* __restrict__ sd,
                               zf* __restrict__ sf, int* __restrict__ flags) {
  const int nk = nf * nf;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)nE * nxy;
       i += (long long)gridDim.x * blockDim.x)
    flags[i] = modes[i].flags;
  const long long n = (long long)nE * nk * nxy;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(i % nxy);
    const long long ek = i / nxy;
    const int k = (int)(ek % nk);
    const int e = (int)(ek / nk);
    const zd v = modes[(long long)e * nxy + m].sig[k];
    sd[i] = v;
    sf[i] = mk<float>((float)v.re, (float)v.im);
  }
}
}  // namespace

hipError_t launch_sigma_tables(iobm_ctx ctx, int nE, const ModeData* modes, zd* sig_d, zf* sig_f, int* flags) {
  const long long n = (long long)nE * ctx->g.nf * ctx->g.nf * ctx->g.nxy;
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_sigma_tables, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, nE, ctx->g.nxy, ctx->g.nf,
                     modes, sig_d, sig_f, flags);
  return hipGetLastError();
}
