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

// r_ij = |U.n| + a + 2 mu / (rho dl) per face, stored as A r / 2.  Interior
// faces take the interface state of Eq. w_interface (its record: U, RT and
// tau = h a / b with a = tau/(tau+h), b = h/(tau+h); mu/rho = tau R T);
// boundary faces take the cell's W^n and the mirrored distance
// dl = 2 (x_f - x_i) . n.  gamma = 5/3.
template <int D>
__global__ void k_imp_rface(Geo g, GasP gas, double h, const double* __restrict__ W, const double* __restrict__ fpar,
                            double* __restrict__ rA) {
  constexpr int MAXF = Cfg<D>::MAXF;
  const int f = blockIdx.x * BLOCK + threadIdx.x;
  if (f >= g.nf) return;
  const int L = g.f_L[f], R = g.f_R[f], sl = g.f_sL[f];
  const size_t so = (size_t)L * MAXF + sl;
  const double area = g.s_sigA[so];           // sigma = +1 on the L side
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
  const double r = fabs(un) + sqrt(5.0 / 3.0 * RT) + 2.0 * nu_over_dl;
  rA[f] = 0.5 * area * r;
}

// Right-hand side -sum_f sigma A F_f^n, diagonal V/dt + sum_f A r / 2, and
// dW = 0.
template <int D>
__global__ void k_imp_rhs(Geo g, const double* __restrict__ F, const double* __restrict__ rA, double* __restrict__ rhs,
                          double* __restrict__ diag, double* __restrict__ dW) {
  constexpr int MAXF = Cfg<D>::MAXF, N = D + 2;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.nc) return;
  const int ns = g.nslot[i];
  double acc[N], dg = 1.0 / g.dtv[i];
  for (int m = 0; m < N; ++m) acc[m] = 0.0;
  for (int s = 0; s < ns; ++s) {
    const int f = g.s_face[i * MAXF + s];
    const double sa = g.s_sigA[i * MAXF + s];
    for (int m = 0; m < N; ++m) acc[m] -= sa * F[(size_t)f * N + m];
    dg += rA[f];
  }
  for (int m = 0; m < N; ++m) {
    rhs[(size_t)i * N + m] = acc[m];
    dW[(size_t)i * N + m] = 0.0;
  }
  diag[i] = dg;
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

// One colour of a PRSGS sweep on Eq. SGS_w: for each cell i of the colour,
// dW_i = (rhs_i - sum_j A/2 [G(W_j + dW_j) - G(W_j)] + sum_j A r/2 dW_j) / diag_i
// over interior neighbours j, with the outward normal of i.
template <int D>
__global__ void k_imp_macro(Geo g, GasP gas, const int* __restrict__ cells, int ncells, const double* __restrict__ W,
                            const double* __restrict__ rA, const double* __restrict__ rhs, const double* __restrict__ diag,
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
    if (j < 0) continue;
    const int f = g.s_face[i * MAXF + s];
    const double sa = g.s_sigA[i * MAXF + s];
    const double sig = g.s_sig[i * MAXF + s];
    const double halfA = 0.5 * (sa * sig);
    double n[D];
    for (int d = 0; d < D; ++d) n[d] = sig * g.f_nrm[(size_t)f * D + d];
    double w0[N], w1[N], dj[N], G0[N], G1[N];
    for (int m = 0; m < N; ++m) {
      w0[m] = W[(size_t)j * N + m];
      dj[m] = dW[(size_t)j * N + m];
      w1[m] = w0[m] + dj[m];
    }
    euler_flux<D>(w1, n, gas.R, G1);
    euler_flux<D>(w0, n, gas.R, G0);
    const double ra = rA[f];
    for (int m = 0; m < N; ++m) {
      acc[m] -= halfA * (G1[m] - G0[m]);
      acc[m] += ra * dj[m];
    }
  }
  const double inv = diag[i];
  for (int m = 0; m < N; ++m) dW[(size_t)i * N + m] = acc[m] / inv;
}

// W~ = W^n + dW into Wn and the target record from W~ (as the explicit
// macro update does from W^{n+1}).
template <int D>
__global__ void k_imp_apply(Geo g, GasP gas, double dt, const double* __restrict__ W, const double* __restrict__ dW,
                            double* __restrict__ Wn, const double* __restrict__ qcur, double* __restrict__ tpar,
                            int* __restrict__ bad) {
  constexpr int N = D + 2;
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= g.nc) return;
  double w[N];
  for (int m = 0; m < N; ++m) {
    w[m] = W[(size_t)i * N + m] + dW[(size_t)i * N + m];
    Wn[(size_t)i * N + m] = w[m];
  }
  target_record<D>(i, w, gas, dt, qcur, tpar, bad);
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
template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void k_imp_micro(Geo g, Leaves L, const int* __restrict__ cells,
                                                     const T* __restrict__ res, T* __restrict__ dphi,
                                                     const double* __restrict__ tpar) {
  constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF;
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
  const double dtt = tpar[(size_t)i * NPAR + P_A], dtv = g.dtv[i];
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
    for (int p = 0; p < P; ++p) dphi[p * cs + o] = (res[p * cs + o] - (T)dtv * off[p]) / (T)dg;
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
