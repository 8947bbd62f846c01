// Implicit step (IUGKS, Sec. 2.3.1-2.3.2 of arXiv 2212.05645): Roe-type
// macroscopic predictor solved by point-relaxation symmetric Gauss-Seidel
// sweeps (Eqs. equ_delw, delta_Flux, Roe, SGS_w) and the upwind microscopic
// increment solved by symmetric Gauss-Seidel sweeps (Eqs. delta_phi,
// SGS_phi).  Both sweep the cells colour by colour: the cells of one colour
// of a greedy colouring of the face-neighbour graph share no face, so one
// launch updates a whole colour and the result is the sequential
// Gauss-Seidel sweep in colour-major cell order.  Interface VDFs, fluxes,
// the target and the closure are those of the explicit step.
// Part of the library's single translation unit, after avs_kernels.hip.

namespace avs {

// r_ij = |U.n| + a + 2 mu / (rho dl) per face.  Interior
// faces take the interface state of Eq. w_interface (its record: U, RT and
// tau = h a / b with a = tau/(tau+h), b = h/(tau+h); mu/rho = tau R T);
// boundary faces take the cell's W^n and the mirrored distance
// dl = 2 (x_f - x_i) . n.  gamma = 5/3.
template <int D>
__global__ void k_imp_rface(Geo g, GasP gas, double h, const double* __restrict__ W, const double* __restrict__ fpar,
                            double* __restrict__ rf) {
  constexpr int MAXF = Cfg<D>::MAXF;
  const int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f >= g.nf) return;
  const int L = g.f_L[f], R = g.f_R[f], sl = g.f_sL[f];
  const size_t so = (size_t)L * MAXF + sl;
  const double* n = g.f_nrm + (size_t)f * D;
  double un = 0.0, RT, nu_over_dl;
  if (R >= 0) {
    const double* par = fpar + (size_t)f * NPAR;
    for (int d = 0; d < D; ++d) un += par[P_U + d] * n[d];
    RT = par[P_RT];
    const double tf = h * par[P_A] / par[P_B];
    double dl2 = 0.0;
    for (int d = 0; d < D; ++d) dl2 += g.s_dx[so * D + d] * g.s_dx[so * D + d];
    nu_over_dl = tf * RT / sqrt(dl2);
  } else {
    double rho, U[D], T;
    prim_from_W<D>(W + (size_t)L * (D + 2), gas, rho, U, T);
    for (int d = 0; d < D; ++d) un += U[d] * n[d];
    RT = gas.R * T;
    double dn = 0.0;
    for (int d = 0; d < D; ++d) dn += g.s_d[so * D + d] * n[d];
    nu_over_dl = tau_of(rho, T, gas) * RT / (2.0 * dn);
  }
  rf[f] = fabs(un) + sqrt(5.0 / 3.0 * RT) + 2.0 * nu_over_dl;
}

// Right-hand side -sum_f sigma A F_f^n, diagonal V/dt + 1/2 sum_f A r, and
// dW = 0.
template <int D, int N = D + 2>
__global__ void k_imp_rhs(Geo g, const double* __restrict__ F, const double* __restrict__ rf, double* __restrict__ rhs,
                          double* __restrict__ diag, double* __restrict__ dW) {
  constexpr int MAXF = Cfg<D>::MAXF;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.nc) return;
  const int ns = g.nslot[i];
  double acc[N], ar = 0.0;
  for (int m = 0; m < N; ++m) acc[m] = 0.0;
  for (int s = 0; s < ns; ++s) {
    const int f = g.s_face[i * MAXF + s];
    const double sa = g.s_sigA[i * MAXF + s];
    for (int m = 0; m < N; ++m) acc[m] -= sa * F[(size_t)f * N + m];
    ar += (sa * g.s_sig[i * MAXF + s]) * rf[f];
  }
  for (int m = 0; m < N; ++m) {
    rhs[(size_t)i * N + m] = acc[m];
    dW[(size_t)i * N + m] = 0.0;
  }
  diag[i] = 1.0 / g.dtv[i] + 0.5 * ar;
}

// Euler flux of W through the unit normal n: (rho U.n, rho U U.n + p n,
// (rho E + p) U.n), p = rho R T.
template <int D>
__device__ __forceinline__ void euler_flux(const double (&w)[D + 2], const double (&n)[D], double R, double (&G)[D + 2]) {
  const double rho = w[0];
  double U[D], uu = 0.0, un = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    U[d] = w[1 + d] / rho;
    uu += U[d] * U[d];
    un += U[d] * n[d];
  }
  const double T = (w[1 + D] - 0.5 * rho * uu) / (1.5 * rho * R);
  const double p = rho * R * T;
  G[0] = rho * un;
#pragma unroll
  for (int d = 0; d < D; ++d) G[1 + d] = rho * U[d] * un + p * n[d];
  G[1 + D] = (w[1 + D] + p) * un;
}

// W reflected in a wall of unit normal n (normal momentum reversed).
template <int D>
__device__ __forceinline__ void mirror_state(const double (&w)[D + 2], const double (&n)[D], double (&o)[D + 2]) {
  double mn = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) mn += w[1 + d] * n[d];
  o[0] = w[0];
#pragma unroll
  for (int d = 0; d < D; ++d) o[1 + d] = w[1 + d] - 2.0 * mn * n[d];
  o[1 + D] = w[1 + D];
}

__device__ __forceinline__ bool wall_face(const Geo& g, int f) {
  const int R = g.f_R[f];
  return R < 0 && g.bc_kind[-1 - R] == 0;
}

// One colour of a PRSGS sweep on Eq. SGS_w: for each cell i of the colour,
// dW_i = (rhs_i - sum_j A/2 [G(W_j + dW_j) - G(W_j)] + sum_j A r/2 dW_j) / diag_i
// over interior neighbours j and wall faces (whose outside is the mirror of
// the cell's own W and current dW), with the outward normal of i; a
// far-field face holds the outside increment at zero.
template <int D>
__global__ void k_imp_macro(Geo g, GasP gas, const int* __restrict__ cells, int ncells, const double* __restrict__ W,
                            const double* __restrict__ rf, const double* __restrict__ rhs, const double* __restrict__ diag,
                            double* __restrict__ dW) {
  constexpr int MAXF = Cfg<D>::MAXF, N = D + 2;
  const int t = blockIdx.x * BLOCK + threadIdx.x;
  if (t >= ncells) return;
  const int i = cells[t];
  const int ns = g.nslot[i];
  double acc[N];
  for (int m = 0; m < N; ++m) acc[m] = rhs[(size_t)i * N + m];
  for (int s = 0; s < ns; ++s) {
    const int j = g.s_nbr[i * MAXF + s];
    const int f = g.s_face[i * MAXF + s];
    if (j < 0 && !wall_face(g, f)) continue;
    const double sa = g.s_sigA[i * MAXF + s];
    const double sig = g.s_sig[i * MAXF + s];
    const double halfA = 0.5 * (sa * sig);
    double n[D];
    for (int d = 0; d < D; ++d) n[d] = sig * g.f_nrm[(size_t)f * D + d];
    double w0[N], w1[N], dj[N], G0[N], G1[N];
    if (j >= 0) {
      for (int m = 0; m < N; ++m) {
        w0[m] = W[(size_t)j * N + m];
        dj[m] = dW[(size_t)j * N + m];
      }
    } else {
      double wi[N], di[N];
      for (int m = 0; m < N; ++m) {
        wi[m] = W[(size_t)i * N + m];
        di[m] = dW[(size_t)i * N + m];
      }
      mirror_state<D>(wi, n, w0);
      mirror_state<D>(di, n, dj);
    }
    for (int m = 0; m < N; ++m) w1[m] = w0[m] + dj[m];
    euler_flux<D>(w1, n, gas.R, G1);
    euler_flux<D>(w0, n, gas.R, G0);
    const double ra = halfA * rf[f];
    for (int m = 0; m < N; ++m) {
      acc[m] -= halfA * (G1[m] - G0[m]);
      acc[m] += ra * dj[m];
    }
  }
  const double inv = diag[i];
  for (int m = 0; m < N; ++m) dW[(size_t)i * N + m] = acc[m] / inv;
}

// Implicit flux of a face, in place over F^n (Eqs. delta_Flux, Roe):
// F_f + 1/2 [G(W_L + dW_L) - G(W_L) + G(W_R + dW_R) - G(W_R)]
// + 1/2 r (dW_L - dW_R) through the face normal, the outside of a boundary
// face as in the predictor (mirror state at a wall, so that no mass crosses
// it; increment 0 at the far field).  The explicit macro update then gives
// W^{n+1} in flux form: exactly conservative after any number of sweeps.
template <int D>
__global__ void k_imp_fhat(Geo g, GasP gas, const double* __restrict__ W, const double* __restrict__ dW,
                           const double* __restrict__ rf, double* __restrict__ F) {
  constexpr int N = D + 2;
  const int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f >= g.nf) return;
  const int L = g.f_L[f], R = g.f_R[f];
  const bool wall = R < 0 && g.bc_kind[-1 - R] == 0;
  double n[D];
  for (int d = 0; d < D; ++d) n[d] = g.f_nrm[(size_t)f * D + d];
  double v[N], w0[N], w1[N], dL[N], G0[N], G1[N];
  for (int m = 0; m < N; ++m) {
    v[m] = F[(size_t)f * N + m];
    w0[m] = W[(size_t)L * N + m];
    dL[m] = dW[(size_t)L * N + m];
    w1[m] = w0[m] + dL[m];
  }
  euler_flux<D>(w1, n, gas.R, G1);
  euler_flux<D>(w0, n, gas.R, G0);
  for (int m = 0; m < N; ++m) v[m] = v[m] + 0.5 * (G1[m] - G0[m]);
  const double hr = 0.5 * rf[f];
  double dR[N];
  if (R >= 0 || wall) {
    if (R >= 0) {
      for (int m = 0; m < N; ++m) {
        w0[m] = W[(size_t)R * N + m];
        dR[m] = dW[(size_t)R * N + m];
      }
    } else {
      double wl[N];
      for (int m = 0; m < N; ++m) wl[m] = W[(size_t)L * N + m];
      mirror_state<D>(wl, n, w0);
      mirror_state<D>(dL, n, dR);
    }
    for (int m = 0; m < N; ++m) w1[m] = w0[m] + dR[m];
    euler_flux<D>(w1, n, gas.R, G1);
    euler_flux<D>(w0, n, gas.R, G0);
    for (int m = 0; m < N; ++m) v[m] = v[m] + 0.5 * (G1[m] - G0[m]);
  } else {
    for (int m = 0; m < N; ++m) dR[m] = 0.0;
  }
  for (int m = 0; m < N; ++m) v[m] = v[m] + hr * (dL[m] - dR[m]);
  for (int m = 0; m < N; ++m) F[(size_t)f * N + m] = v[m];
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK, (waves_hint<D, T>())) void k_passC_res(Geo g, Leaves L, VGrid vg,
                                                                          const T* __restrict__ vin,
                                                                          const T* __restrict__ fv, T* __restrict__ res,
                                                                          const double* __restrict__ fpar,
                                                                          const double* __restrict__ tpar,
                                                                          const double* __restrict__ lam) {
  d_passC<D, T, true>(g, L, vg, vin, fv, res, fpar, tpar, lam, nullptr, nullptr, blockIdx.x);
}

// x[p][i][k] = 0 for every component and leaf k < n of cell i = block.
template <typename T>
__global__ void k_imp_zero(int P, int nc, Leaves L, T* __restrict__ x) {
  const int i = blockIdx.x;
  const size_t cs = (size_t)nc * L.ld;
  for (int k = threadIdx.x; k < L.n; k += BLOCK)
    for (int p = 0; p < P; ++p) x[p * cs + (size_t)i * L.ld + k] = (T)0;
}

// One colour of a symmetric Gauss-Seidel sweep on Eq. SGS_phi, scaled by
// dt/V: per leaf, dphi_i = (res_i - dt/V sum_{xi.n<0} sigma A xi.n dphi_j)
// / (1 + dt/tau~ + dt/V sum_{xi.n>=0} sigma A xi.n), res the right-hand side
// from pass C.  Boundary faces hold the outside increment at zero.
// P components; dt/tau~ of cell i is tpar[i * tstride + toff].  With out
// (the cell's last visit of the last sweep, when its increment is final),
// also out = vin + dphi; out may be the buffer of res, which only the cell
// itself reads.
template <int D, typename T, int P = Cfg<D>::P>
__global__ __launch_bounds__(BLOCK) void k_imp_micro(Geo g, Leaves L, const int* __restrict__ cells,
                                                     const T* res, T* __restrict__ dphi,
                                                     const double* __restrict__ tpar, int tstride, int toff,
                                                     const T* __restrict__ vin = nullptr, T* out = nullptr) {
  constexpr int MAXF = Cfg<D>::MAXF;
  __shared__ double snrm[MAXF][D];
  __shared__ double ssa[MAXF];
  __shared__ int snbr[MAXF];
  const int i = cells[blockIdx.x];
  const int ns = g.nslot[i];
  if (threadIdx.x < MAXF) {
    const int s = threadIdx.x;
    const int f = s < ns ? g.s_face[i * MAXF + s] : 0;
    snbr[s] = s < ns ? g.s_nbr[i * MAXF + s] : -1;
    ssa[s] = s < ns ? g.s_sigA[i * MAXF + s] : 0.0;
    for (int d = 0; d < D; ++d) snrm[s][d] = g.f_nrm[(size_t)f * D + d];
  }
  __syncthreads();
  const double dtt = tpar[(size_t)i * tstride + toff], dtv = g.dtv[i];
  const size_t cs = (size_t)g.nc * L.ld;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    leaf_load<D>(L, k, xi, A, u);
    double dg = 1.0 + dtt;
    T off[P];
#pragma unroll
    for (int p = 0; p < P; ++p) off[p] = 0;
    for (int s = 0; s < ns; ++s) {
      const double w = ssa[s] * normal_speed<D>(xi, snrm[s]);
      if (w >= 0.0) {
        dg += dtv * w;
      } else if (snbr[s] >= 0) {
        const size_t o = (size_t)snbr[s] * L.ld + k;
#pragma unroll
        for (int p = 0; p < P; ++p) off[p] += (T)w * dphi[p * cs + o];
      }
    }
    const size_t o = (size_t)i * L.ld + k;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const T x = (res[p * cs + o] - (T)dtv * off[p]) / (T)dg;
      dphi[p * cs + o] = x;
      if (out) out[p * cs + o] = vin[p * cs + o] + x;
    }
  }
}

// phi^{n+1} = phi^n + dphi, in place over dphi.
template <typename T>
__global__ void k_imp_finish(int P, int nc, Leaves L, const T* __restrict__ vin, T* __restrict__ x) {
  const int i = blockIdx.x;
  const size_t cs = (size_t)nc * L.ld;
  for (int k = threadIdx.x; k < L.n; k += BLOCK)
    for (int p = 0; p < P; ++p) {
      const size_t o = p * cs + (size_t)i * L.ld + k;
      x[o] = vin[o] + x[o];
    }
}

}  // namespace avs

namespace avs {

// ------------------------------------------- Rykov diatomic equilibrium
// g^phi = (1 - 1/Z) phi^t + (1/Z) phi^r for phi = G, H, R (Eqs. GHR_equ,
// equ11-equ13) at every leaf, for one state per block: st = (rho, U[D],
// T_t, T_r, q_t[D], q_r[D]).  T = (3 T_t + 2 T_r)/5, p_t = rho R T_t,
// p = rho R T; H carries the 3 - D hidden translational degrees of freedom
// (zero in 3-D).  Out: [3][n][ld] in T.
struct RykovP {
  double R, Z, delta, omega0, omega1;
};

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void k_rykov_eq(Leaves L, VGrid vg, RykovP gp, int n, const double* __restrict__ states,
                                                   T* __restrict__ out) {
  // the two Maxwellians (at T_t and at T) from separable per-axis tables of
  // the half-finest grid (exact products of one-dimensional factors)
  extern __shared__ double lds_d[];
  double* tabt = lds_d;
  double* tabr = lds_d + D * vg.numax;
  __shared__ double part[NPAR], parr[NPAR];
  const int i = blockIdx.x;
  if (i >= n) return;
  const double* st = states + (size_t)i * (3 + 3 * D);
  const double rho = st[0], Tt = st[1 + D], Tr = st[2 + D];
  double U[D], qt[D], qr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    U[d] = st[1 + d];
    qt[d] = st[3 + D + d];
    qr[d] = st[3 + 2 * D + d];
  }
  const double R = gp.R;
  const double Teq = (3.0 * Tt + 2.0 * Tr) / 5.0;
  const double RTt = R * Tt, RT = R * Teq;
  const double pt = rho * RTt, p = rho * RT;
  if (threadIdx.x == 0) {
    part[P_COEF] = rho * pow(2.0 * M_PI * RTt, -0.5 * D);
    parr[P_COEF] = rho * pow(2.0 * M_PI * RT, -0.5 * D);
    for (int d = 0; d < 3; ++d) {
      part[P_U + d] = d < D ? U[d] : 0.0;
      parr[P_U + d] = d < D ? U[d] : 0.0;
    }
    part[P_I2RT] = 0.5 / RTt;
    parr[P_I2RT] = 0.5 / RT;
  }
  __syncthreads();
  build_tab<D>(tabt, part, vg);
  build_tab<D>(tabr, parr, vg);
  __syncthreads();
  const double wt = 1.0 - 1.0 / gp.Z, wr = 1.0 / gp.Z;
  const double kt = 1.0 / (15.0 * pt * RTt), kr = gp.omega0 / (15.0 * p * RT);
  const double irt_t = 1.0 / RTt, irt = 1.0 / RT;
  const double mt = (1.0 - gp.delta) / (pt * RTt), mr = gp.omega1 * (1.0 - gp.delta) / (p * RT);
  const double RTr = R * Tr;
  const size_t cs = (size_t)n * L.ld;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    leaf_load<D>(L, k, xi, A, u);
    double c2 = 0.0, cqt = 0.0, cqr = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double c = xi[d] - U[d];
      c2 += c * c;
      cqt += c * qt[d];
      cqr += c * qr[d];
    }
    const double gt = maxw<D>(part, tabt, vg.numax, u);
    const double g = maxw<D>(parr, tabr, vg.numax, u);
    const double at = cqt * kt, ar = cqt * kr;
    const double Gt = gt * (1.0 + at * (c2 * irt_t - D - 2));
    const double Gr = g * (1.0 + ar * (c2 * irt - D - 2));
    const double Ht = RTt * gt * (3 - D) * (1.0 + at * (c2 * irt_t - D));
    const double Hr = RT * g * (3 - D) * (1.0 + ar * (c2 * irt - D));
    const double Rt = RTr * (Gt + mt * cqr * gt);
    const double Rr = RT * (Gr + mr * cqr * g);
    const size_t o = (size_t)i * L.ld + k;
    out[o] = (T)(wt * Gt + wr * Gr);
    out[cs + o] = (T)(wt * Ht + wr * Hr);
    out[2 * cs + o] = (T)(wt * Rt + wr * Rr);
  }
}

}  // namespace avs
