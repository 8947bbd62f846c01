// Explicit step of the Rykov diatomic model (Sec. 2.3 in its explicit limit
// with the equilibrium of Eqs. GHR_equ, equ11-equ13 and the rotational
// source of Eq. equ19), two-dimensional, FP64, on a fixed velocity tree.
// Three reduced distributions per cell and leaf, [3][cell][leaf]: G, H (the
// hidden translational degree of freedom) and R (rotational energy, two
// degrees of freedom); five conserved variables (rho, rho U, rho E,
// rho E_rot).  One pass per stage, written for clarity rather than speed:
//   k_dg_recon   limited least-squares reconstruction at x_f - xi h into the
//                interface rows (boundary Maxwellian triples on incoming leaves)
//   k_dg_face    interface moments, rotational and heat-flux relaxation over h,
//                Rykov equilibrium, characteristic blend in place, flux F_f
//   k_dg_macro   W* = W - dt/V sum sigma A F, point-implicit rotational exchange
//   k_dg_target  closure coefficients of the Rykov target (5 x 5 system)
//   k_dg_update  flux divergence, relaxation, heat fluxes of phi^{n+1}
// Part of the library's single translation unit, after avs_kernels.hip.

namespace avs {

constexpr int DG_N = 5;      // rho, rho U (2), rho E, rho E_rot
constexpr int DG_NT = 12;    // target record: rho, U0, U1, T_t, T_r, qt0, qt1, qr0, qr1, dt/tau, E_rot target, T

struct DiaGas {
  double R, Z, delta, omega0, omega1;
};

// Rykov equilibrium triple at one leaf (c = xi - U), or, with t_only, the
// translational part at (T_t, T_r) with zero heat fluxes.
// gt and g are the Maxwellians at T_t and at T = (3 T_t + 2 T_r)/5.
__device__ __forceinline__ void dg_equilibrium(const DiaGas& gp, double rho, const double (&c)[2], double Tt, double Tr,
                                               const double* qt, const double* qr, bool t_only, double gt, double g,
                                               double& G, double& H, double& Rr) {
  const double R = gp.R;
  const double T = (3.0 * Tt + 2.0 * Tr) / 5.0;
  const double c2 = c[0] * c[0] + c[1] * c[1];
  const double RTt = R * Tt, RT = R * T;
  if (t_only) {
    G = gt;
    H = RTt * gt;
    Rr = R * Tr * gt;
    return;
  }
  const double cqt = c[0] * qt[0] + c[1] * qt[1], cqr = c[0] * qr[0] + c[1] * qr[1];
  const double pt = rho * RTt, p = rho * RT;
  const double at = cqt / (15.0 * pt * RTt), ar = gp.omega0 * cqt / (15.0 * p * RT);
  const double Gt = gt * (1.0 + at * (c2 / RTt - 4.0));
  const double Gr = g * (1.0 + ar * (c2 / RT - 4.0));
  const double Ht = RTt * gt * (1.0 + at * (c2 / RTt - 2.0));
  const double Hr = RT * g * (1.0 + ar * (c2 / RT - 2.0));
  const double Rt = R * Tr * (Gt + (1.0 - gp.delta) * cqr / (pt * RTt) * gt);
  const double Rq = RT * (Gr + gp.omega1 * (1.0 - gp.delta) * cqr / (p * RT) * g);
  const double wt = 1.0 - 1.0 / gp.Z, wr = 1.0 / gp.Z;
  G = wt * Gt + wr * Gr;
  H = wt * Ht + wr * Hr;
  Rr = wt * Rt + wr * Rq;
}

// Separable per-axis tables of the Maxwellians at T_t and at T (the
// half-finest grid carries every leaf centre), built by the whole block
// from a record r = (rho, U0, U1, T_t, T_r, ...); followed by a barrier.
__device__ __forceinline__ void dg_tables(const double* r, double R, const VGrid& vg, double* tabt, double* tabr,
                                          double* part, double* parr) {
  if (threadIdx.x == 0) {
    const double Tt = r[3], T = (3.0 * r[3] + 2.0 * r[4]) / 5.0;
    part[P_COEF] = r[0] / (2.0 * M_PI * R * Tt);
    parr[P_COEF] = r[0] / (2.0 * M_PI * R * T);
    for (int d = 0; d < 3; ++d) part[P_U + d] = parr[P_U + d] = d < 2 ? r[1 + d] : 0.0;
    part[P_I2RT] = 0.5 / (R * Tt);
    parr[P_I2RT] = 0.5 / (R * T);
  }
  __syncthreads();
  build_tab<2>(tabt, part, vg);
  build_tab<2>(tabr, parr, vg);
  __syncthreads();
}

// rho, U, T_t, T_r, T from W = (rho, rho U, rho E, rho E_rot).
__device__ __forceinline__ bool dg_temps(const double* w, double R, double& rho, double (&U)[2], double& Tt, double& Tr,
                                         double& T) {
  rho = w[0];
  U[0] = w[1] / rho;
  U[1] = w[2] / rho;
  Tr = w[4] / (rho * R);
  Tt = (w[3] - 0.5 * rho * (U[0] * U[0] + U[1] * U[1]) - w[4]) / (1.5 * rho * R);
  T = (3.0 * Tt + 2.0 * Tr) / 5.0;
  return rho > 0.0 && Tt > 0.0 && Tr > 0.0;
}

// moments (rho, rho U, rho E, rho E_rot) contribution of one leaf
__device__ __forceinline__ void dg_mom(double* m, double A, const double (&xi)[2], double G, double H, double Rr) {
  const double xi2 = xi[0] * xi[0] + xi[1] * xi[1];
  m[0] += A * G;
  m[1] += A * G * xi[0];
  m[2] += A * G * xi[1];
  m[3] += A * (0.5 * (xi2 * G + H) + Rr);
  m[4] += A * Rr;
}

// Venkatakrishnan psi for one face, the same branches as its definition
// divided through by D2 (and, for eps = 0, through t = D2/D1 or 1/t).
__device__ __forceinline__ double dg_psi(double d1, double d2, double eps2) {
  if (d2 == 0.0) return 1.0;
  if (eps2 > 0.0) return (d1 * d1 + eps2 + 2.0 * d1 * d2) / (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2);
  if (fabs(d2) <= fabs(d1)) {
    const double t = d2 / d1;
    return (1.0 + 2.0 * t) / (1.0 + t + 2.0 * t * t);
  }
  const double u = d1 / d2;
  return u * (u + 2.0) / (u * u + u + 2.0);
}

__global__ __launch_bounds__(BLOCK) void k_dg_recon(Geo g, Leaves L, double h, const double* __restrict__ vin,
                                                   double* __restrict__ fv, DiaGas gp) {
  constexpr int MAXF = MAXF2;
  const int i = blockIdx.x;
  const int ns = g.nslot[i];
  const size_t cs = (size_t)g.nc * L.ld, fs = (size_t)g.nf * L.ld;
  // neighbour rows (a slot without an interior neighbour reads the cell's
  // own row and is skipped), so that every load of a leaf is issued before
  // any is used
  size_t nb[MAXF];
  unsigned mask = 0;
#pragma unroll
  for (int s = 0; s < MAXF; ++s) {
    const int j = s < ns ? g.s_nbr[i * MAXF + s] : -1;
    if (j >= 0) mask |= 1u << s;
    nb[s] = (size_t)(j >= 0 ? j : i) * L.ld;
  }
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[2], A;
    int u[2];
    leaf_load<2>(L, k, xi, A, u);
    double ph[3], gr[3][2], pmax[3], pmin[3], nv[MAXF][3];
#pragma unroll
    for (int p = 0; p < 3; ++p) ph[p] = vin[p * cs + (size_t)i * L.ld + k];
#pragma unroll
    for (int s = 0; s < MAXF; ++s)
#pragma unroll
      for (int p = 0; p < 3; ++p) nv[s][p] = vin[p * cs + nb[s] + k];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      gr[p][0] = gr[p][1] = 0.0;
      pmax[p] = pmin[p] = ph[p];
    }
#pragma unroll
    for (int s = 0; s < MAXF; ++s) {
      if (!(mask & (1u << s))) continue;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const double v = nv[s][p];
        const double dv = v - ph[p];
        gr[p][0] += dv * g.s_lsq[(size_t)(i * MAXF + s) * 2];
        gr[p][1] += dv * g.s_lsq[(size_t)(i * MAXF + s) * 2 + 1];
        pmax[p] = fmax(pmax[p], v);
        pmin[p] = fmin(pmin[p], v);
      }
    }
    const double eps2 = g.eps2[i];
    double lg[3][2];
    for (int p = 0; p < 3; ++p) {
      double lim = ns > 0 ? INFINITY : 1.0;
      for (int s = 0; s < ns; ++s) {
        const double* d = g.s_d + (size_t)(i * MAXF + s) * 2;
        const double d2 = gr[p][0] * d[0] + gr[p][1] * d[1];
        const double d1 = d2 > 0.0 ? pmax[p] - ph[p] : pmin[p] - ph[p];
        lim = fmin(lim, dg_psi(d1, d2, eps2));
      }
      lg[p][0] = lim * gr[p][0];
      lg[p][1] = lim * gr[p][1];
    }
    for (int s = 0; s < ns; ++s) {
      const int f = g.s_face[i * MAXF + s];
      const double sig = g.s_sig[i * MAXF + s];
      const double sn = normal_speed<2>(xi, g.f_nrm + (size_t)f * 2);
      const bool upwind = sig > 0.0 ? sn >= 0.0 : sn < 0.0;
      const int Rc = g.f_R[f];
      const size_t o = (size_t)f * L.ld + k;
      if (upwind) {
        const double* d = g.s_d + (size_t)(i * MAXF + s) * 2;
        const double r0 = d[0] - xi[0] * h, r1 = d[1] - xi[1] * h;
        for (int p = 0; p < 3; ++p) fv[p * fs + o] = ph[p] + (lg[p][0] * r0 + lg[p][1] * r1);
      } else if (Rc < 0) {
        // incoming leaf of a boundary face: the equilibrium triple of the
        // wall (unit density, scaled by the wall density later) or of the far field
        const int b = -1 - Rc;
        const double* st = g.bc_prim + (size_t)b * 4;
        const double rho = g.bc_kind[b] == 0 ? 1.0 : st[0];
        const double c[2] = {xi[0] - st[1], xi[1] - st[2]};
        const double RT = gp.R * st[3];
        const double gv = rho / (2.0 * M_PI * RT) * exp(-(c[0] * c[0] + c[1] * c[1]) / (2.0 * RT));
        fv[o] = gv;
        fv[fs + o] = RT * gv;
        fv[2 * fs + o] = RT * gv;
      }
    }
  }
}

// block sum of n doubles per thread into red (LDS), result in red[0..n)
template <int NN>
__device__ __forceinline__ void dg_sum(double* v, double* red) {
  for (int m = 0; m < NN; ++m) {
    double x = v[m];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o);
    if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * NN + m] = x;
  }
  __syncthreads();
  if (threadIdx.x < NN) {
    double x = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) x += red[w * NN + threadIdx.x];
    red[BLOCK / 64 * NN + threadIdx.x] = x;
  }
  __syncthreads();
  for (int m = 0; m < NN; ++m) v[m] = red[BLOCK / 64 * NN + m];
  __syncthreads();
}

__global__ __launch_bounds__(BLOCK) void k_dg_face(Geo g, Leaves L, VGrid vg, GasP vgas, DiaGas gp, double h,
                                                  double* __restrict__ fv, double* __restrict__ F, int* __restrict__ bad) {
  extern __shared__ double lds_d[];
  __shared__ double red[(BLOCK / 64 + 1) * 8];
  __shared__ double rec[16], part[NPAR], parr[NPAR];
  const int f = blockIdx.x;
  const int Rc = g.f_R[f];
  const size_t fs = (size_t)g.nf * L.ld;
  const double n[2] = {g.f_nrm[(size_t)f * 2], g.f_nrm[(size_t)f * 2 + 1]};
  double* row0 = fv + (size_t)f * L.ld;
  if (Rc >= 0) {
    double m[5] = {0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < L.n; k += BLOCK) {
      double xi[2], A;
      int u[2];
      leaf_load<2>(L, k, xi, A, u);
      dg_mom(m, A, xi, row0[k], row0[fs + k], row0[2 * fs + k]);
    }
    dg_sum<5>(m, red);
    double rho, U[2], Ttb, Trb, T;
    const bool ok = dg_temps(m, gp.R, rho, U, Ttb, Trb, T);
    double q[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < L.n; k += BLOCK) {
      double xi[2], A;
      int u[2];
      leaf_load<2>(L, k, xi, A, u);
      const double c0 = xi[0] - U[0], c1 = xi[1] - U[1], c2 = c0 * c0 + c1 * c1;
      const double Gv = row0[k], Hv = row0[fs + k], Rv = row0[2 * fs + k];
      const double et = A * 0.5 * (c2 * Gv + Hv), er = A * Rv;
      q[0] += et * c0;
      q[1] += et * c1;
      q[2] += er * c0;
      q[3] += er * c1;
    }
    dg_sum<4>(q, red);
    if (threadIdx.x == 0) {
      if (!ok) atomicMin(bad, g.nc + f);
      const double tf = ok ? tau_of(rho, Ttb, vgas) : 1.0;
      const double kz = h / (gp.Z * tf);
      const double ER = (m[4] + kz * (rho * gp.R * T)) / (1.0 + kz);
      const double Tr = ER / (rho * gp.R);
      const double Tt = Ttb + (2.0 / 3.0) * (Trb - Tr);
      const double lt = (1.0 - 1.0 / gp.Z) / 3.0 + gp.omega0 / (3.0 * gp.Z);
      const double lr = (1.0 - gp.delta) * ((1.0 - 1.0 / gp.Z) * Tr / Tt + gp.omega1 / gp.Z);
      rec[0] = rho;
      rec[1] = U[0];
      rec[2] = U[1];
      rec[3] = Tt;
      rec[4] = Tr;
      rec[5] = q[0] / (1.0 + (1.0 - lt) * h / tf);
      rec[6] = q[1] / (1.0 + (1.0 - lt) * h / tf);
      rec[7] = q[2] / (1.0 + (1.0 - lr) * h / tf);
      rec[8] = q[3] / (1.0 + (1.0 - lr) * h / tf);
      rec[9] = tf / (tf + h);
      rec[10] = h / (tf + h);
    }
    __syncthreads();
    double* tabt = lds_d;
    double* tabr = lds_d + 2 * vg.numax;
    dg_tables(rec, gp.R, vg, tabt, tabr, part, parr);
    double fl[5] = {0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < L.n; k += BLOCK) {
      double xi[2], A;
      int u[2];
      leaf_load<2>(L, k, xi, A, u);
      const double c[2] = {xi[0] - rec[1], xi[1] - rec[2]};
      double Ge, He, Re;
      dg_equilibrium(gp, rec[0], c, rec[3], rec[4], rec + 5, rec + 7, false, maxw<2>(part, tabt, vg.numax, u),
                     maxw<2>(parr, tabr, vg.numax, u), Ge, He, Re);
      const double Gv = rec[9] * row0[k] + rec[10] * Ge;
      const double Hv = rec[9] * row0[fs + k] + rec[10] * He;
      const double Rv = rec[9] * row0[2 * fs + k] + rec[10] * Re;
      row0[k] = Gv;
      row0[fs + k] = Hv;
      row0[2 * fs + k] = Rv;
      dg_mom(fl, A * normal_speed<2>(xi, n), xi, Gv, Hv, Rv);
    }
    dg_sum<5>(fl, red);
    if (threadIdx.x < 5) F[(size_t)f * 5 + threadIdx.x] = fl[threadIdx.x];
    return;
  }
  const int b = -1 - Rc;
  const bool wall = g.bc_kind[b] == 0;
  double sc = 1.0;
  if (wall) {
    double nd[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < L.n; k += BLOCK) {
      double xi[2], A;
      int u[2];
      leaf_load<2>(L, k, xi, A, u);
      const double s = normal_speed<2>(xi, n);
      if (s > 0.0) nd[0] += A * s * row0[k];
      if (s < 0.0) nd[1] += A * (-s) * row0[k];
    }
    dg_sum<2>(nd, red);
    sc = nd[0] / nd[1];
  }
  double fl[5] = {0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[2], A;
    int u[2];
    leaf_load<2>(L, k, xi, A, u);
    const double s = normal_speed<2>(xi, n);
    double Gv = row0[k], Hv = row0[fs + k], Rv = row0[2 * fs + k];
    if (wall && s < 0.0) {
      Gv *= sc;
      Hv *= sc;
      Rv *= sc;
      row0[k] = Gv;
      row0[fs + k] = Hv;
      row0[2 * fs + k] = Rv;
    }
    dg_mom(fl, A * s, xi, Gv, Hv, Rv);
  }
  dg_sum<5>(fl, red);
  if (threadIdx.x < 5) F[(size_t)f * 5 + threadIdx.x] = fl[threadIdx.x];
}

// W* = W - dt/V sum sigma A F; rotational exchange point-implicit with tau
// of W*; target record of W^{n+1} with the heat fluxes q of phi^n.
__global__ void k_dg_macro(Geo g, GasP vgas, DiaGas gp, double dt, const double* __restrict__ F,
                           const double* __restrict__ W, double* __restrict__ Wn, const double* __restrict__ q,
                           double* __restrict__ tp, int* __restrict__ bad) {
  constexpr int MAXF = MAXF2;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.nc) return;
  double Fs[5] = {0, 0, 0, 0, 0};
  for (int s = 0; s < g.nslot[i]; ++s) {
    const int f = g.s_face[i * MAXF + s];
    const double sa = g.s_sigA[i * MAXF + s];
    for (int m = 0; m < 5; ++m) Fs[m] += sa * F[(size_t)f * 5 + m];
  }
  double w[5];
  const double dtv = g.dtv[i];
  for (int m = 0; m < 5; ++m) w[m] = W[(size_t)i * 5 + m] - dtv * Fs[m];
  double rho, U[2], Tt, Tr, T;
  if (!dg_temps(w, gp.R, rho, U, Tt, Tr, T)) {
    atomicMin(bad, i);
    rho = 1.0; Tt = Tr = T = 1.0;
  }
  const double tt = tau_of(rho, Tt, vgas);
  const double k = dt / (gp.Z * tt);
  w[4] = (w[4] + k * (rho * gp.R * T)) / (1.0 + k);
  for (int m = 0; m < 5; ++m) Wn[(size_t)i * 5 + m] = w[m];
  dg_temps(w, gp.R, rho, U, Tt, Tr, T);
  double* r = tp + (size_t)i * DG_NT;
  r[0] = rho;
  r[1] = U[0];
  r[2] = U[1];
  r[3] = Tt;
  r[4] = Tr;
  for (int d = 0; d < 4; ++d) r[5 + d] = q[(size_t)i * 4 + d];
  r[9] = dt / tt;
  r[10] = (1.0 - 1.0 / gp.Z) * w[4] + rho * gp.R * T / gp.Z;
  r[11] = T;
}

// Closure coefficients: the Rykov target (or, with init, the translational
// part with zero heat fluxes) plus sum_m lambda_m e_m has the moments
// target = (rho, rho U, rho E, E_rot target) of W; e_m = (1, c, |c|^2) x
// (g, R T g, R T g) at T and (0, 0, R T g).
__global__ __launch_bounds__(BLOCK) void k_dg_target(Geo g, Leaves L, VGrid vg, DiaGas gp, const double* __restrict__ tp,
                                                    const double* __restrict__ Wt, double* __restrict__ lam, int init,
                                                    int* __restrict__ bad) {
  extern __shared__ double lds_d[];
  __shared__ double red[(BLOCK / 64 + 1) * 32];
  __shared__ double Jm[25], bv[5], xv[5], part[NPAR], parr[NPAR];
  const int i = blockIdx.x;
  const double* r = tp + (size_t)i * DG_NT;
  double* tabt = lds_d;
  double* tabr = lds_d + 2 * vg.numax;
  dg_tables(r, gp.R, vg, tabt, tabr, part, parr);
  const double rho = r[0], U[2] = {r[1], r[2]}, Tt = r[3], Tr = r[4], T = r[11];
  const double RT = gp.R * T;
  double acc[30];
  for (int m = 0; m < 30; ++m) acc[m] = 0.0;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[2], A;
    int u[2];
    leaf_load<2>(L, k, xi, A, u);
    const double c[2] = {xi[0] - U[0], xi[1] - U[1]};
    const double gv = maxw<2>(parr, tabr, vg.numax, u);
    double Ge, He, Re;
    dg_equilibrium(gp, rho, c, Tt, Tr, r + 5, r + 7, init != 0, maxw<2>(part, tabt, vg.numax, u), gv, Ge, He, Re);
    dg_mom(acc, A, xi, Ge, He, Re);
    const double bs[4] = {1.0, c[0], c[1], c[0] * c[0] + c[1] * c[1]};
    for (int e = 0; e < 4; ++e) dg_mom(acc + 5 + 5 * e, A, xi, bs[e] * gv, RT * bs[e] * gv, RT * bs[e] * gv);
    dg_mom(acc + 25, A, xi, 0.0, 0.0, RT * gv);
  }
  // reduce 30 sums in groups of 8 (the LDS buffer holds 32 per wave)
  for (int g0 = 0; g0 < 30; g0 += 8) {
    double v[8];
    for (int m = 0; m < 8; ++m) v[m] = g0 + m < 30 ? acc[g0 + m] : 0.0;
    dg_sum<8>(v, red);
    for (int m = 0; m < 8; ++m)
      if (g0 + m < 30) acc[g0 + m] = v[m];
  }
  if (threadIdx.x == 0) {
    for (int l = 0; l < 5; ++l) {
      for (int e = 0; e < 5; ++e) Jm[l * 5 + e] = acc[5 + 5 * e + l];
      const double tgt = l < 4 ? Wt[(size_t)i * 5 + l] : (init ? Wt[(size_t)i * 5 + 4] : r[10]);
      bv[l] = tgt - acc[l];
    }
    if (!solve_small<5>(Jm, bv, xv)) atomicMin(bad, i);
    for (int e = 0; e < 5; ++e) lam[(size_t)i * 5 + e] = xv[e];
  }
}

// phi^{n+1} = (phi^n + dt/tau g~ - dt/V sum sigma A xi.n phi_f) / (1 + dt/tau),
// or with init the closed initial state; heat fluxes of the result about U.
__global__ __launch_bounds__(BLOCK) void k_dg_update(Geo g, Leaves L, VGrid vg, DiaGas gp, const double* __restrict__ vin,
                                                    const double* __restrict__ fv, double* __restrict__ vout,
                                                    const double* __restrict__ tp, const double* __restrict__ lam,
                                                    double* __restrict__ q, int init) {
  constexpr int MAXF = MAXF2;
  extern __shared__ double lds_d[];
  __shared__ double red[(BLOCK / 64 + 1) * 8];
  __shared__ double part[NPAR], parr[NPAR];
  const int i = blockIdx.x;
  const double* r = tp + (size_t)i * DG_NT;
  double* tabt = lds_d;
  double* tabr = lds_d + 2 * vg.numax;
  dg_tables(r, gp.R, vg, tabt, tabr, part, parr);
  const double rho = r[0], U[2] = {r[1], r[2]}, Tt = r[3], Tr = r[4], T = r[11], dtt = r[9];
  const double RT = gp.R * T, dtv = g.dtv[i];
  double la[5];
  for (int e = 0; e < 5; ++e) la[e] = lam[(size_t)i * 5 + e];
  const int ns = g.nslot[i];
  const size_t cs = (size_t)g.nc * L.ld, fs = (size_t)g.nf * L.ld;
  double qa[4] = {0, 0, 0, 0};
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[2], A;
    int u[2];
    leaf_load<2>(L, k, xi, A, u);
    const double c[2] = {xi[0] - U[0], xi[1] - U[1]};
    const double c2 = c[0] * c[0] + c[1] * c[1];
    const double gv = maxw<2>(parr, tabr, vg.numax, u);
    double Ge, He, Re;
    dg_equilibrium(gp, rho, c, Tt, Tr, r + 5, r + 7, init != 0, maxw<2>(part, tabt, vg.numax, u), gv, Ge, He, Re);
    const double poly = la[0] + la[1] * c[0] + la[2] * c[1] + la[3] * c2;
    const double tg[3] = {Ge + poly * gv, He + poly * RT * gv, Re + poly * RT * gv + la[4] * RT * gv};
    double nv[3];
    if (init) {
      for (int p = 0; p < 3; ++p) nv[p] = tg[p];
    } else {
      double div[3] = {0, 0, 0};
      for (int s = 0; s < ns; ++s) {
        const int f = g.s_face[i * MAXF + s];
        const double w = g.s_sigA[i * MAXF + s] * normal_speed<2>(xi, g.f_nrm + (size_t)f * 2);
        for (int p = 0; p < 3; ++p) div[p] += w * fv[p * fs + (size_t)f * L.ld + k];
      }
      for (int p = 0; p < 3; ++p)
        nv[p] = (vin[p * cs + (size_t)i * L.ld + k] + dtt * tg[p] - dtv * div[p]) / (1.0 + dtt);
    }
    for (int p = 0; p < 3; ++p) vout[p * cs + (size_t)i * L.ld + k] = nv[p];
    const double et = A * 0.5 * (c2 * nv[0] + nv[1]), er = A * nv[2];
    qa[0] += et * c[0];
    qa[1] += et * c[1];
    qa[2] += er * c[0];
    qa[3] += er * c[1];
  }
  dg_sum<4>(qa, red);
  if (threadIdx.x < 4) q[(size_t)i * 4 + threadIdx.x] = qa[threadIdx.x];
}

// Initial target record from W (no exchange, zero heat fluxes).
__global__ void k_dg_initrec(int nc, DiaGas gp, const double* __restrict__ W, double* __restrict__ tp,
                             int* __restrict__ bad) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
  double rho, U[2], Tt, Tr, T;
  if (!dg_temps(W + (size_t)i * 5, gp.R, rho, U, Tt, Tr, T)) atomicMin(bad, i);
  double* r = tp + (size_t)i * DG_NT;
  r[0] = rho;
  r[1] = U[0];
  r[2] = U[1];
  r[3] = Tt;
  r[4] = Tr;
  for (int d = 0; d < 4; ++d) r[5 + d] = 0.0;
  r[9] = 0.0;
  r[10] = W[(size_t)i * 5 + 4];
  r[11] = T;
}

// Heat fluxes q_t, q_r of the state about the U of the record tp.
__global__ __launch_bounds__(BLOCK) void k_dg_heat(Geo g, Leaves L, const double* __restrict__ v,
                                                  const double* __restrict__ tp, double* __restrict__ q) {
  __shared__ double red[(BLOCK / 64 + 1) * 8];
  const int i = blockIdx.x;
  const double U0 = tp[(size_t)i * DG_NT + 1], U1 = tp[(size_t)i * DG_NT + 2];
  const size_t cs = (size_t)g.nc * L.ld;
  double qa[4] = {0, 0, 0, 0};
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[2], A;
    int u[2];
    leaf_load<2>(L, k, xi, A, u);
    const size_t o = (size_t)i * L.ld + k;
    const double c0 = xi[0] - U0, c1 = xi[1] - U1, c2 = c0 * c0 + c1 * c1;
    const double et = A * 0.5 * (c2 * v[o] + v[cs + o]), er = A * v[2 * cs + o];
    qa[0] += et * c0;
    qa[1] += et * c1;
    qa[2] += er * c0;
    qa[3] += er * c1;
  }
  dg_sum<4>(qa, red);
  if (threadIdx.x < 4) q[(size_t)i * 4 + threadIdx.x] = qa[threadIdx.x];
}

// --------------------------------------------- adaptation of the state
// Criterion partials over groups of CRIT_CELLS cells: M1 = A G / rho,
// M2 = A (1/2 (|c|^2 G + H) + R) / (rho E - rho |U|^2/2), max over the group,
// in a fixed operation order (no contraction) so that the flags are
// reproducible bit for bit.
__global__ __launch_bounds__(BLOCK) void k_dg_crit_partial(Leaves L, int nc, const double* __restrict__ vdf,
                                                          const double* __restrict__ W, double* __restrict__ part) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  const int grp = blockIdx.y;
  if (k >= L.n) return;
  const size_t cs = (size_t)nc * L.ld;
  double xi[2], A;
  int u[2];
  leaf_load<2>(L, k, xi, A, u);
  double m = -INFINITY;
  const int i1 = min(nc, (grp + 1) * CRIT_CELLS);
  for (int i = grp * CRIT_CELLS; i < i1; ++i) {
    const double* w = W + (size_t)i * DG_N;
    const double rho = w[0];
    const double U0 = w[1] / rho, U1 = w[2] / rho;
    double ke = U0 * U0;
    ke = ke + U1 * U1;
    const double eint = w[3] - 0.5 * rho * ke;
    double c = xi[0] - U0;
    double c2 = c * c;
    c = xi[1] - U1;
    c2 = c2 + c * c;
    const size_t o = (size_t)i * L.ld + k;
    const double G = vdf[o], H = vdf[cs + o], Rr = vdf[2 * cs + o];
    const double M1 = (A * G) / rho;
    const double M2 = (A * (0.5 * (c2 * G + H) + Rr)) / eint;
    m = fmax(m, fmax(M1, M2));
  }
  part[(size_t)grp * L.cap + k] = m;
}

// Consanguinity reconstruction of G, H, R onto the new leaves: a kept or
// split leaf copies its source, a merged parent is the balanced pairwise
// mean ((f0 + f1) + (f2 + f3)) / 4 of its children.
__global__ __launch_bounds__(BLOCK) void k_dg_gather(int nc, Leaves Lo, Leaves Ln, const int* __restrict__ kind,
                                                    const int* __restrict__ src, const double* __restrict__ vin,
                                                    double* __restrict__ vout) {
#pragma clang fp contract(off)
  const int i = blockIdx.x;
  const size_t cso = (size_t)nc * Lo.ld, csn = (size_t)nc * Ln.ld;
  for (int j = threadIdx.x; j < Ln.n; j += BLOCK) {
    const int k = src[j];
    for (int p = 0; p < 3; ++p) {
      const double* a = vin + p * cso + (size_t)i * Lo.ld;
      double v;
      if (kind[j] == 2) v = ((a[k] + a[k + 1]) + (a[k + 2] + a[k + 3])) * 0.25;
      else v = a[k];
      vout[p * csn + (size_t)i * Ln.ld + j] = v;
    }
  }
}

// Closure of the state onto W in place: f + sum_m lambda_m e_m with the
// directions of the target's closure at T of W.
__global__ __launch_bounds__(BLOCK) void k_dg_close(Geo g, Leaves L, VGrid vg, DiaGas gp, const double* __restrict__ W,
                                                   double* __restrict__ v, int* __restrict__ bad) {
  extern __shared__ double lds_d[];
  __shared__ double red[(BLOCK / 64 + 1) * 32];
  __shared__ double Jm[25], bv[5], xv[5], part[NPAR], parr[NPAR], rec[5];
  const int i = blockIdx.x;
  if (threadIdx.x == 0) {
    double rho, U[2], Tt, Tr, T;
    if (!dg_temps(W + (size_t)i * DG_N, gp.R, rho, U, Tt, Tr, T)) atomicMin(bad, i);
    rec[0] = rho; rec[1] = U[0]; rec[2] = U[1]; rec[3] = Tt; rec[4] = Tr;
  }
  __syncthreads();
  double* tabt = lds_d;
  double* tabr = lds_d + 2 * vg.numax;
  dg_tables(rec, gp.R, vg, tabt, tabr, part, parr);
  const double rho = rec[0], U[2] = {rec[1], rec[2]};
  const double RT = gp.R * (3.0 * rec[3] + 2.0 * rec[4]) / 5.0;
  const size_t cs = (size_t)g.nc * L.ld;
  double acc[30];
  for (int m = 0; m < 30; ++m) acc[m] = 0.0;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[2], A;
    int u[2];
    leaf_load<2>(L, k, xi, A, u);
    const size_t o = (size_t)i * L.ld + k;
    dg_mom(acc, A, xi, v[o], v[cs + o], v[2 * cs + o]);
    const double c[2] = {xi[0] - U[0], xi[1] - U[1]};
    const double gv = maxw<2>(parr, tabr, vg.numax, u);
    const double bs[4] = {1.0, c[0], c[1], c[0] * c[0] + c[1] * c[1]};
    for (int e = 0; e < 4; ++e) dg_mom(acc + 5 + 5 * e, A, xi, bs[e] * gv, RT * bs[e] * gv, RT * bs[e] * gv);
    dg_mom(acc + 25, A, xi, 0.0, 0.0, RT * gv);
  }
  for (int g0 = 0; g0 < 30; g0 += 8) {
    double vv[8];
    for (int m = 0; m < 8; ++m) vv[m] = g0 + m < 30 ? acc[g0 + m] : 0.0;
    dg_sum<8>(vv, red);
    for (int m = 0; m < 8; ++m)
      if (g0 + m < 30) acc[g0 + m] = vv[m];
  }
  if (threadIdx.x == 0) {
    for (int l = 0; l < 5; ++l) {
      for (int e = 0; e < 5; ++e) Jm[l * 5 + e] = acc[5 + 5 * e + l];
      bv[l] = W[(size_t)i * DG_N + l] - acc[l];
    }
    if (!solve_small<5>(Jm, bv, xv)) atomicMin(bad, i);
  }
  __syncthreads();
  const double l0 = xv[0], l1 = xv[1], l2 = xv[2], l3 = xv[3], l4 = xv[4];
  (void)rho;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[2], A;
    int u[2];
    leaf_load<2>(L, k, xi, A, u);
    const double c[2] = {xi[0] - U[0], xi[1] - U[1]};
    const double gv = maxw<2>(parr, tabr, vg.numax, u);
    const double poly = l0 + l1 * c[0] + l2 * c[1] + l3 * (c[0] * c[0] + c[1] * c[1]);
    const size_t o = (size_t)i * L.ld + k;
    v[o] = v[o] + poly * gv;
    v[cs + o] = v[cs + o] + poly * RT * gv;
    v[2 * cs + o] = v[2 * cs + o] + (poly * RT * gv + l4 * RT * gv);
  }
}

}  // namespace avs
