// Adjoint gradient of the total transmission with respect to V(r).
//
// A depends on V only through -diag(V), so d psi_mu / d V_r = A^-1 (e_r psi_mu(r)).
// The transmitted amplitudes are linear functionals t_nu,mu = l_nu^T psi_mu
// (the readout: l_nu = (1/Nxy) exp(-i G_nu . r) lr_nu[i] on the far planes),
// and T_mu = sum_nu (v_nu / v_mu) |t_nu,mu|^2, hence
//     dT_tot / dV(r) = 2 Re sum_{E,mu} lambda_mu(r) psi_mu(r),
//     lambda_mu = sum_nu C_nu,mu W_nu,  A W_nu = l_nu,  C_nu,mu = (v_nu / v_mu) conj(t_nu,mu),
// using A^T = A (one extra solve per outgoing channel with the same operator).
// W_nu and psi_mu are combinations of real-lateral-basis solutions w_b, u_a
// (cos/sin standing waves), so per energy the gradient is the bilinear form
//     g(r) = 2 Re sum_{b,a} D[b][a] w_b(r) u_a(r),  D = Q^T C P,
// with P (psi from u) and Q (W from w) the +-i combination coefficients.
#include "internal.h"

namespace {

// Adjoint right-hand side l_nu in the real lateral basis: on the far planes
// (plane nz-nf+i for left incidence, nf-1-i for right incidence)
//   g(plane, r) = (1/Nxy) lr_nu[i] trig(G_nu . r),  trig = cos (kind 1) / sin (kind 2).
__global__ void k_rhs_adjoint(int nx, int ny, int nz, int nf, const int* __restrict__ e_rhs,
                              const int* __restrict__ mode_rhs, const int* __restrict__ kind_rhs, int side,
                              const ModeData* __restrict__ modes, zd* __restrict__ b) {
  const int rhs = blockIdx.y;
  const int nxy = nx * ny;
  const long long vol = (long long)nxy * nz;
  const int m = mode_rhs[rhs];
  const int kind = kind_rhs[rhs];
  if (m < 0 || m >= nxy) return;  // ids are validated on the host
  const ModeData& md = modes[(long long)e_rhs[rhs] * nxy + m];
  const int ix = m % nx, iy = m / nx;
  const int nux = ix < nx / 2 ? ix : ix - nx;
  const int nuy = iy < ny / 2 ? iy : iy - ny;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < vol;
       idx += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(idx / nxy);
    const int p = (int)(idx - (long long)z * nxy);
    const int i = side ? nf - 1 - z : z - (nz - nf);
    zd val = mk(0.0, 0.0);
    if (i >= 0 && i < nf) {
      const int jj = p / nx, ii = p - jj * nx;
      long long a = ((long long)nux * ii) % nx;
      long long bb = ((long long)nuy * jj) % ny;
      double ph = 2.0 * M_PI * ((double)a / nx + (double)bb / ny);
      double s, c;
      sincos(ph, &s, &c);
      double trig = kind == 2 ? s : c;
      val = (trig / nxy) * md.lr[i];
    }
    b[rhs * vol + idx] = val;
  }
}

// D[b][a] for every basis pair of one energy.  Basis index k of the energy
// maps to at most two channels (the +-G pair) with coefficients:
//   forward  psi_mu = sum_a P[mu][a] u_a   (P = 1 for cos, i*sgn_mu for sin)
//   adjoint  W_nu   = sum_b Q[nu][b] w_b   (Q = 1 for cos, -i*sgn_nu for sin)
// chan[k][0..1] = request ids (or -1), coef[k][0..1] = the coefficient of
// basis k in those channels.
struct GradD {
  int nxy;
  const int* base;      // [nE+1] first basis index of each energy
  const int* chan;      // [nbasis][2] request ids
  const zd* pcoef;      // [nbasis][2] P coefficient (forward)
  const zd* qcoef;      // [nbasis][2] Q coefficient (adjoint)
  const int* req_mode;  // [nreq]
  const int* req_e;     // [nreq]
  const ModeData* modes;
  const zd* tamp;       // [nreq][nxy] outgoing amplitudes t[nu] of request mu
  zd* D;                // [nE] blocks, each [n_e][n_e], offset = dbase[e]
  const long long* dbase;
};

__global__ void k_grad_D(GradD G) {
  const int e = blockIdx.y;
  const int b0 = G.base[e], n = G.base[e + 1] - b0;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n * n) return;
  const int bi = tid / n, ai = tid - bi * n;  // D[b][a]
  const int kb = b0 + bi, ka = b0 + ai;
  const ModeData* md = G.modes + (long long)e * G.nxy;
  zd acc = mk(0.0, 0.0);
  for (int s = 0; s < 2; ++s) {
    const int cnu = G.chan[2 * kb + s];
    if (cnu < 0) continue;
    const int nu = G.req_mode[cnu];
    const zd q = G.qcoef[2 * kb + s];
    for (int u = 0; u < 2; ++u) {
      const int cmu = G.chan[2 * ka + u];
      if (cmu < 0) continue;
      const int mu = G.req_mode[cmu];
      const zd p = G.pcoef[2 * ka + u];
      const zd t = G.tamp[(long long)cmu * G.nxy + nu];
      const double w = md[nu].v / md[mu].v;
      acc = acc + q * (w * conj(t)) * p;
    }
  }
  G.D[G.dbase[e] + (long long)bi * n + ai] = acc;
}

// g(r) = 2 Re sum_e sum_{b,a} D_e[b][a] w_b(r) u_a(r)
__global__ void k_grad(long long vol, int nE, const int* __restrict__ base, const long long* __restrict__ dbase,
                       const zd* __restrict__ D, const zd* __restrict__ u, const zd* __restrict__ w,
                       double* __restrict__ g) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < vol;
       r += (long long)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int e = 0; e < nE; ++e) {
      const int b0 = base[e], n = base[e + 1] - b0;
      const zd* De = D + dbase[e];
      for (int a = 0; a < n; ++a) {
        zd s = mk(0.0, 0.0);
        for (int b = 0; b < n; ++b) s = s + De[(long long)b * n + a] * w[(long long)(b0 + b) * vol + r];
        const zd ua = u[(long long)(b0 + a) * vol + r];
        acc += s.re * ua.re - s.im * ua.im;
      }
    }
    g[r] = 2.0 * acc;
  }
}

}  // namespace

hipError_t launch_rhs_adjoint(iobm_ctx c, int nrhs, const int* e_rhs, const int* mode_rhs, const int* kind_rhs,
                              int side, const ModeData* modes, zd* b) {
  long long vol = c->g.npts;
  long long bx = (vol + 255) / 256;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(k_rhs_adjoint, dim3((unsigned)bx, nrhs), dim3(256), 0, c->stream, c->g.nx, c->g.ny, c->g.nz,
                     c->g.nf, e_rhs, mode_rhs, kind_rhs, side, modes, b);
  return hipGetLastError();
}

hipError_t launch_grad_D(iobm_ctx c, int nE, int nmax, const int* base, const int* chan, const zd* pcoef,
                         const zd* qcoef, const int* req_mode, const int* req_e, const ModeData* modes,
                         const zd* tamp, zd* D, const long long* dbase) {
  GradD G;
  G.nxy = c->g.nxy;
  G.base = base; G.chan = chan; G.pcoef = pcoef; G.qcoef = qcoef;
  G.req_mode = req_mode; G.req_e = req_e; G.modes = modes; G.tamp = tamp; G.D = D; G.dbase = dbase;
  int n2 = nmax * nmax;
  hipLaunchKernelGGL(k_grad_D, dim3((n2 + 127) / 128, nE), dim3(128), 0, c->stream, G);
  return hipGetLastError();
}

hipError_t launch_grad(iobm_ctx c, int nE, const int* base, const long long* dbase, const zd* D, const zd* u,
                       const zd* w, double* g) {
  long long vol = c->g.npts;
  long long bx = (vol + 255) / 256;
  if (bx > 4096) bx = 4096;
  hipLaunchKernelGGL(k_grad, dim3((unsigned)bx), dim3(256), 0, c->stream, vol, nE, base, dbase, D, u, w, g);
  return hipGetLastError();
}
