// HIP kernels of the global adaptive-velocity-space sweep (gfx950).
//
// Layout: vdf[comp][cell][leaf], leaf fastest, row stride L.ld.  One
// workgroup of 256 threads (4 wave64) owns one physical cell and streams its
// velocity row in chunks of 256 consecutive leaves, so every VDF access is a
// coalesced 256-element segment and all per-cell data are wave-uniform.
// Maxwellians are evaluated from separable per-axis exponential tables held
// in LDS: every leaf centre lies on the half-finest grid of the velocity box,
// so exp(-|xi-U|^2/2RT) = prod_d t_d[u_d] with t_d tabulated once per
// face/cell instead of one exp per (cell, leaf).
#include "avs_internal.h"

// Minimum waves per SIMD requested for the two streaming passes, per form
// (FP64 kernels keep their registers, FP32 kernels ask for occupancy).
#ifndef AVS_WAVES_F64
#define AVS_WAVES_F64 1
#endif
#ifndef AVS_WAVES_F32
#define AVS_WAVES_F32 4
#endif

namespace avs {

template <int D, typename T>
constexpr int waves_hint() { return (D == 3 || sizeof(T) == 8) ? AVS_WAVES_F64 : AVS_WAVES_F32; }

template <typename T>
__device__ __forceinline__ double ld_(const T* p) { return (double)(*p); }

// Element at a 32-bit byte offset from a workgroup-uniform row pointer: the
// offset stays in one vector register and the row pointer in scalar
// registers (no per-lane 64-bit address arithmetic).  Rows are < 4 GiB.
template <typename T>
__device__ __forceinline__ T at_(const T* row, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + off);
}
template <typename T>
__device__ __forceinline__ T* ptr_at_(T* row, unsigned off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(row) + off);
}

template <int D>
struct Cfg {
  static constexpr int P = (D == 2) ? 2 : 1;
  static constexpr int MAXF = (D == 2) ? MAXF2 : MAXF3;
  static constexpr int NM = (D == 2) ? NM2 : NM3;
  static constexpr int NS = (D + 2) * (D + 3) / 2;   // symmetric Gram entries
};

// Workgroups are dealt to the 8 XCDs round-robin by linear id.  Block x of a
// grid of round_up(nc, 8) blocks takes position (x % 8) * ceil(nc/8) + x / 8
// of the locality order of the cells (a space-filling curve through the cell
// centres), so each XCD walks a compact patch of the mesh and neighbouring
// cells share its L2.  Returns -1 for the padding blocks.
__device__ __forceinline__ int xcd_cell(const Geo& g, int x) {
  const int per = (g.nc + 7) >> 3;
  const int i = (x & 7) * per + (x >> 3);
  return i < g.nc ? g.order[i] : -1;
}

// ---------------------------------------------------------------- reductions
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
#pragma unroll
  for (int m = 0; m < N; ++m) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[m] += __shfl_xor(v[m], o);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < N; ++m) red[w * N + m] = v[m];
  }
  __syncthreads();
  // one entry's four partials at a time: the empty asm that takes the sum
  // as an operand, with a memory clobber, forms each total before the next
  // entry is read (otherwise all 4N reads are issued at once and the sums
  // sunk past the barrier: for N = 25 that held 200 registers and set the
  // occupancy of the whole kernel)
#pragma unroll
  for (int m = 0; m < N; ++m) {
    v[m] = (red[m] + red[N + m]) + (red[2 * N + m] + red[3 * N + m]);
    __asm__ volatile("" : "+v"(v[m]) : : "memory");
  }
  __syncthreads();
}

// Block total of each of N per-thread values, returned to thread t < N for
// entry t (other threads get 0); the same association as block_sum.
template <int N>
__device__ __forceinline__ double block_sum_pick(double (&v)[N], double* red) {
#pragma unroll
  for (int m = 0; m < N; ++m) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[m] += __shfl_xor(v[m], o);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < N; ++m) red[w * N + m] = v[m];
  }
  __syncthreads();
  const int t = threadIdx.x;
  const double r = t < N ? (red[t] + red[N + t]) + (red[2 * N + t] + red[3 * N + t]) : 0.0;
  __syncthreads();
  return r;
}

// ------------------------------------------------------------- equilibria
template <int D>
__device__ __forceinline__ void build_tab(double* tab, const double* par, const VGrid& vg) {
  const double i2rt = par[P_I2RT];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double x0 = vg.x0[d], hh = vg.hh[d], U = par[P_U + d];
    for (int u = threadIdx.x; u < vg.numax; u += BLOCK) {
      const double c = (x0 + u * hh) - U;
      tab[d * vg.numax + u] = exp(-(c * c) * i2rt);
    }
  }
}

template <int D>
__device__ __forceinline__ double maxw(const double* par, const double* tab, int numax, const int (&u)[D]) {
  double g = par[P_COEF];
#pragma unroll
  for (int d = 0; d < D; ++d) g *= tab[d * numax + u[d]];
  return g;
}

// Shakhov pair (G, H) from the Maxwellian value g (Eqs. equ14-equ17, K = 0).
template <int D>
__device__ __forceinline__ void shakhov(const double* par, double g, const double (&xi)[D], double& G, double& H) {
  double c2 = 0.0, cq = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double c = xi[d] - par[P_U + d];
    c2 += c * c;
    cq += c * par[P_Q + d];
  }
  const double sk = par[P_SHK] * cq, irt = par[P_IRT];
  G = g + sk * (c2 * irt - (D + 2)) * g;
  if (D == 2) {
    const double rtg = par[P_RT] * g;
    H = rtg + sk * (c2 * irt - D) * rtg;
  } else {
    H = 0.0;
  }
}

// Compute-type variants used by the sweep kernels: R = double in the FP64
// form, float in the FP32 form (records stay FP64 in memory and are
// converted once per workgroup).
template <int D, typename R>
__device__ __forceinline__ void build_tab_r(R* tab, const double* par, const VGrid& vg) {
  const double i2rt = par[P_I2RT];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double x0 = vg.x0[d], hh = vg.hh[d], U = par[P_U + d];
    for (int u = threadIdx.x; u < vg.numax; u += BLOCK) {
      const double c = (x0 + u * hh) - U;
      tab[d * vg.numax + u] = (R)exp(-(c * c) * i2rt);
    }
  }
}

template <int D, typename R>
__device__ __forceinline__ R maxw_r(const R* par, const R* tab, int numax, const int (&u)[D]) {
  R g = par[P_COEF];
#pragma unroll
  for (int d = 0; d < D; ++d) g *= tab[d * numax + u[d]];
  return g;
}

template <int D, typename R>
__device__ __forceinline__ void shakhov_r(const R* par, R g, const R (&xi)[D], R& G, R& H) {
  R c2 = 0, cq = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const R c = xi[d] - par[P_U + d];
    c2 += c * c;
    cq += c * par[P_Q + d];
  }
  const R sk = par[P_SHK] * cq, irt = par[P_IRT];
  G = g + sk * (c2 * irt - (R)(D + 2)) * g;
  if (D == 2) {
    const R rtg = par[P_RT] * g;
    H = rtg + sk * (c2 * irt - (R)D) * rtg;
  } else {
    H = 0;
  }
}

// Fill an NPAR record from conserved W (cell target or face state).
template <int D>
__device__ __forceinline__ bool prim_from_W(const double* W, const GasP& gas, double& rho, double (&U)[D], double& T) {
  rho = W[0];
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    U[d] = W[1 + d] / rho;
    ke += U[d] * U[d];
  }
  T = (W[1 + D] - 0.5 * rho * ke) / (1.5 * rho * gas.R);
  return rho > 0.0 && T > 0.0;
}

template <int D>
__device__ __forceinline__ void eq_record(double* par, double rho, const double (&U)[D], double T, const double* q,
                                          const GasP& gas) {
  const double RT = gas.R * T;
  par[P_COEF] = rho * pow(2.0 * M_PI * RT, -0.5 * D);
#pragma unroll
  for (int d = 0; d < 3; ++d) par[P_U + d] = d < D ? U[d] : 0.0;
  par[P_RT] = RT;
  par[P_I2RT] = 0.5 / RT;
  par[P_IRT] = 1.0 / RT;
#pragma unroll
  for (int d = 0; d < 3; ++d) par[P_Q + d] = (d < D && q) ? q[d] : 0.0;
  par[P_SHK] = gas.model == 1 ? (1.0 - gas.Pr) / (5.0 * rho * RT * RT) : 0.0;
}

// tau = mu(T) / p (Eq. equ3): VHS power law, or Sutherland's law (Eq.
// Sutherland) with the reference state in place of the freestream.
__device__ __forceinline__ double tau_of(double rho, double T, const GasP& gas) {
  const double mu = gas.law == 1
                        ? gas.mu_ref * pow(T / gas.T_ref, 1.5) * (gas.T_ref + gas.C_s) / (T + gas.C_s)
                        : gas.mu_ref * pow(T / gas.T_ref, gas.omega);
  return mu / (rho * gas.R * T);
}

// Solve J x = b ((D+2)x(D+2)) by Gaussian elimination with partial pivoting.
template <int N>
__device__ bool solve_small(double* J, double* b, double* x) {
  // J (row-major N x N), b and x in LDS, one thread: the loops are not
  // unrolled, so the solve costs the kernel no registers (held in registers
  // it bounded the occupancy of the whole per-cell kernel)
#pragma unroll 1
  for (int c = 0; c < N; ++c) {
    int p = c;
    double best = fabs(J[c * N + c]);
#pragma unroll 1
    for (int r = c + 1; r < N; ++r)
      if (fabs(J[r * N + c]) > best) { best = fabs(J[r * N + c]); p = r; }
    if (!(best > 0.0)) return false;
    if (p != c) {
#pragma unroll 1
      for (int k = 0; k < N; ++k) { double t = J[c * N + k]; J[c * N + k] = J[p * N + k]; J[p * N + k] = t; }
      double t = b[c]; b[c] = b[p]; b[p] = t;
    }
#pragma unroll 1
    for (int r = c + 1; r < N; ++r) {
      const double f = J[r * N + c] / J[c * N + c];
#pragma unroll 1
      for (int k = c; k < N; ++k) J[r * N + k] -= f * J[c * N + k];
      b[r] -= f * b[c];
    }
  }
#pragma unroll 1
  for (int r = N - 1; r >= 0; --r) {
    double s = b[r];
#pragma unroll 1
    for (int k = r + 1; k < N; ++k) s -= J[r * N + k] * x[k];
    x[r] = s / J[r * N + r];
  }
  return true;
}

// Gram matrix of the equilibrium directions: S = sum_k A_k b_a b_b g_k with
// b = (1, c_1..c_D, |c|^2) about the record's U (accumulated per node).
template <int D>
__device__ __forceinline__ void gram_acc(double* S, double Ag, const double (&c)[D], double c2) {
  double b[D + 2];
  b[0] = 1.0;
#pragma unroll
  for (int d = 0; d < D; ++d) b[1 + d] = c[d];
  b[D + 1] = c2;
  int m = 0;
#pragma unroll
  for (int a = 0; a < D + 2; ++a) {
#pragma unroll
    for (int e = a; e < D + 2; ++e) S[m++] += Ag * b[a] * b[e];
  }
}

// J_lm = M_l[e_m] for e_m = (b_m g, (3-D) RT b_m g), from S (see closure).
// S holds the upper triangle of the symmetric Gram matrix row by row; J is
// written row-major (N x N, N = D + 2).
template <int D>
__device__ __forceinline__ int sym_index(int a, int e) {
  if (a > e) { const int t = a; a = e; e = t; }
  return a * (D + 2) - a * (a - 1) / 2 + (e - a);
}

template <int D>
__device__ void gram_to_J(const double* S, const double* par, double* J) {
  constexpr int N = D + 2;
  double U2 = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) U2 += par[P_U + d] * par[P_U + d];
  const double hidden = (D == 2) ? par[P_RT] : 0.0;
#pragma unroll 1
  for (int c = 0; c < N; ++c) {
    const double s0 = S[sym_index<D>(0, c)];
    J[c] = s0;
    double e = 0.5 * S[sym_index<D>(D + 1, c)] + 0.5 * (U2 + hidden) * s0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double sd = S[sym_index<D>(1 + d, c)];
      J[(1 + d) * N + c] = sd + par[P_U + d] * s0;
      e += par[P_U + d] * sd;
    }
    J[(D + 1) * N + c] = e;
  }
}

// LDS work space of the one-thread closure solve of a per-cell kernel.
template <int D>
struct ClosureWork {
  double S[Cfg<D>::NS], J[(D + 2) * (D + 2)], b[D + 2], x[D + 2];
};

// s = xi . n as the ordered sum of products without contraction: its sign
// picks the upwind side, so it must be reproducible bit for bit.
template <int D>
__device__ __forceinline__ double normal_speed(const double (&xi)[D], const double* n) {
#pragma clang fp contract(off)
  double s = xi[0] * n[0];
#pragma unroll
  for (int d = 1; d < D; ++d) s = s + xi[d] * n[d];
  return s;
}

// xi . n where it only weighs a flux (no side is chosen from it): fused
// multiply-adds, one instruction fewer per dimension than normal_speed.
template <int D>
__device__ __forceinline__ double flux_weight(const double (&xi)[D], const double* n) {
  double s = xi[0] * n[0];
#pragma unroll
  for (int d = 1; d < D; ++d) s = fma(xi[d], n[d], s);
  return s;
}

// Moment contribution sum A (G, xi G, (|xi|^2 G + H)/2).
template <int D>
__device__ __forceinline__ void mom_acc(double* M, double A, const double (&xi)[D], double xi2, double G, double H) {
  const double aG = A * G;
  M[0] += aG;
#pragma unroll
  for (int d = 0; d < D; ++d) M[1 + d] += aG * xi[d];
  M[D + 1] += 0.5 * A * (xi2 * G + H);
}

template <int D>
__device__ __forceinline__ void leaf_load(const Leaves& L, int k, double (&xi)[D], double& A, int (&u)[D]) {
#pragma unroll
  for (int d = 0; d < D; ++d) {
    xi[d] = at_(L.xi + (size_t)d * L.cap, (unsigned)k * 8u);
    u[d] = at_(L.u + (size_t)d * L.cap, (unsigned)k * 4u);
  }
  A = at_(L.w, (unsigned)k * 8u);
}

// The same from the per-dimension row pointers: each load a scalar base
// plus the lane offset (in the kernels whose scalar registers have room:
// face_eq and the target; pass A and pass C run out of them).
template <int D>
__device__ __forceinline__ void leaf_load_rows(const Leaves& L, int k, double (&xi)[D], double& A, int (&u)[D]) {
#pragma unroll
  for (int d = 0; d < D; ++d) {
    xi[d] = at_(L.xd[d], (unsigned)k * 8u);
    u[d] = at_(L.ud[d], (unsigned)k * 4u);
  }
  A = at_(L.w, (unsigned)k * 8u);
}

// ---------------------------------------------------------- leaf geometry
// xi = lo + (idx + 1/2) h_l, A = prod h_l, h_l = (hi - lo)/(base 2^l); the
// operation order matches the oracle exactly (no contraction) so that the
// criterion can be compared bit for bit.
template <int D>
__global__ void k_leaf_geom(int n, int cap, const int* __restrict__ level, const int* __restrict__ idx,
                            int* __restrict__ u, double* __restrict__ xi, double* __restrict__ w, VGrid vg,
                            int lmax, int b0, int b1, int b2, double lo0, double lo1, double lo2, double hi0,
                            double hi1, double hi2) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= n) return;
  const int l = level[k];
  const int base[3] = {b0, b1, b2};
  const double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
  double a = 1.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double h = (hi[d] - lo[d]) / (double)(base[d] << l);
    const int ix = idx[d * cap + k];
    xi[d * cap + k] = lo[d] + ((double)ix + 0.5) * h;
    u[d * cap + k] = (2 * ix + 1) << (lmax - l);
    a = (d == 0) ? h : a * h;
  }
  w[k] = a;
}

// ------------------------------------------------ initial state / closure
// phi = closure(g_eq(W), W): discrete Maxwellian corrected along its own
// equilibrium directions so that its moments equal W.
template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void k_init_vdf(Geo g, Leaves L, VGrid vg, GasP gas, const double* __restrict__ W,
                                                     T* __restrict__ vdf, int* __restrict__ bad, int close) {
  constexpr int N = D + 2, NS = Cfg<D>::NS;
  extern __shared__ double lds[];
  double* tab = lds;
  double* red = lds + D * vg.numax;
  __shared__ double par[NPAR];
  __shared__ double lam[N];
  __shared__ ClosureWork<D> cw;
  const int i = blockIdx.x;
  if (threadIdx.x == 0) {
    double rho, U[D], T_;
    if (!prim_from_W<D>(W + (size_t)i * N, gas, rho, U, T_)) atomicMin(bad, i);
    eq_record<D>(par, rho, U, T_, nullptr, gas);
  }
  __syncthreads();
  build_tab<D>(tab, par, vg);
  __syncthreads();
  if (close) {
    double acc[N + NS];
#pragma unroll
    for (int m = 0; m < N + NS; ++m) acc[m] = 0.0;
    for (int k = threadIdx.x; k < L.n; k += BLOCK) {
      double xi[D], A;
      int u[D];
      leaf_load<D>(L, k, xi, A, u);
      const double gv = maxw<D>(par, tab, vg.numax, u);
      double c[D], c2 = 0.0, xi2 = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) { c[d] = xi[d] - par[P_U + d]; c2 += c[d] * c[d]; xi2 += xi[d] * xi[d]; }
      mom_acc<D>(acc, A, xi, xi2, gv, D == 2 ? par[P_RT] * gv : 0.0);
      gram_acc<D>(acc + N, A * gv, c, c2);
    }
    block_sum<N + NS>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int m = 0; m < NS; ++m) cw.S[m] = acc[N + m];
      gram_to_J<D>(cw.S, par, cw.J);
#pragma unroll
      for (int m = 0; m < N; ++m) cw.b[m] = W[(size_t)i * N + m] - acc[m];
      if (!solve_small<N>(cw.J, cw.b, cw.x)) atomicMin(bad, i);
      for (int m = 0; m < N; ++m) lam[m] = cw.x[m];
    }
  } else if (threadIdx.x < N) {
    lam[threadIdx.x] = 0.0;     // the discrete Maxwellian as it is
  }
  __syncthreads();
  const size_t cs = (size_t)g.nc * L.ld;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    leaf_load<D>(L, k, xi, A, u);
    const double gv = maxw<D>(par, tab, vg.numax, u);
    double c2 = 0.0, poly = lam[0];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double c = xi[d] - par[P_U + d];
      c2 += c * c;
      poly += lam[1 + d] * c;
    }
    poly += lam[D + 1] * c2;
    const double G = gv + poly * gv;
    vdf[(size_t)i * L.ld + k] = (T)G;
    if (D == 2) vdf[cs + (size_t)i * L.ld + k] = (T)(par[P_RT] * G);
  }
}

// ------------------------------------------------------- cell moments / q
// M[phi_i] and q_i = 1/2 sum A c (c^2 G + H), c = xi - U(W_i) (Eqs. updat_W, equ8).
// One leaf's share of a cell's moments (rho, m, rho E) and heat flux q
// about U: acc[0..N) and acc[N..N+D).
template <int D>
__device__ __forceinline__ void state_mom_acc(double* acc, const double (&xi)[D], double A, const double (&U)[D],
                                              double G, double H) {
  constexpr int N = D + 2;
  double xi2 = 0.0, c[D], c2 = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) { xi2 += xi[d] * xi[d]; c[d] = xi[d] - U[d]; c2 += c[d] * c[d]; }
  mom_acc<D>(acc, A, xi, xi2, G, H);
  const double e = 0.5 * A * (c2 * G + H);
#pragma unroll
  for (int d = 0; d < D; ++d) acc[N + d] += e * c[d];
}

template <int D, typename T>
__device__ __forceinline__ void d_cell_moments(Geo g, Leaves L, const T* __restrict__ vdf,
                                               const double* __restrict__ W, double* __restrict__ mom,
                                               double* __restrict__ q, int bx) {
  constexpr int N = D + 2;
  __shared__ double red[4 * (N + D)];
  const int i = bx;
  const size_t cs = (size_t)g.nc * L.ld;
  double U[D];
#pragma unroll
  for (int d = 0; d < D; ++d) U[d] = W[(size_t)i * N + 1 + d] / W[(size_t)i * N];
  double acc[N + D];
#pragma unroll
  for (int m = 0; m < N + D; ++m) acc[m] = 0.0;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    leaf_load<D>(L, k, xi, A, u);
    const double G = ld_(vdf + (size_t)i * L.ld + k);
    const double H = (D == 2) ? ld_(vdf + cs + (size_t)i * L.ld + k) : 0.0;
    state_mom_acc<D>(acc, xi, A, U, G, H);
  }
  block_sum<N + D>(acc, red);
  if (threadIdx.x == 0) {
    for (int m = 0; m < N; ++m) mom[(size_t)i * N + m] = acc[m];
    for (int d = 0; d < D; ++d) q[(size_t)i * D + d] = acc[N + d];
  }
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void k_cell_moments(Geo g, Leaves L, const T* __restrict__ vdf,
                             const double* __restrict__ W, double* __restrict__ mom, double* __restrict__ q) {
  d_cell_moments<D, T>(g, L, vdf, W, mom, q, blockIdx.x);
}

// ------------------------------------------------- limited gradient (S2-S3)
// The stencil of one cell, loaded once per workgroup: row pointers of the
// cell and of its neighbours (the cell's own row for a boundary face, whose
// difference is then zero), least-squares coefficients and face offsets.
template <int D, typename T>
struct Stencil {
  static constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF;
  // 3-D: the LSQ coefficients and face offsets stay in LDS and are read
  // where they are used (held in scalar registers, the six faces' constants
  // spilled and were reloaded lane by lane on every leaf)
  static constexpr bool kLds = D == 3;
  int ns;
  unsigned nbmask;            // bit s: face s has an interior neighbour
  const T* own[P];
  const T* nb[MAXF][P];
  T cf[kLds ? 1 : MAXF][D];
  T dd[kLds ? 1 : MAXF][D];
  const T* lcf = nullptr;
  const T* ldd = nullptr;
  T eps2;
  __device__ __forceinline__ T CF(int s, int d) const {
    if constexpr (kLds) return lcf[s * D + d]; else return cf[s][d];
  }
  __device__ __forceinline__ T DD(int s, int d) const {
    if constexpr (kLds) return ldd[s * D + d]; else return dd[s][d];
  }
};

// The per-cell constants come from global memory (uniform loads, scalar
// registers) or, with lcf/ldd non-null, from LDS: copied to vector registers
// in 2-D FP32 (registers to spare), read at their use in 3-D (Stencil::kLds,
// which needs lcf/ldd).
template <int D, typename T>
__device__ __forceinline__ void load_stencil(const Geo& g, const T* __restrict__ vdf, size_t cs, int ld, int c,
                                             Stencil<D, T>& st, const T* lcf = nullptr, const T* ldd = nullptr) {
  constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF;
  st.ns = g.nslot[c];
  st.nbmask = 0;
  st.eps2 = (T)g.eps2[c];
#pragma unroll
  for (int p = 0; p < P; ++p) st.own[p] = vdf + p * cs + (size_t)c * ld;
#pragma unroll
  for (int s = 0; s < MAXF; ++s) {
    const int j = s < st.ns ? g.s_nbr[c * MAXF + s] : -1;
    if (j >= 0) st.nbmask |= 1u << s;
#pragma unroll
    for (int p = 0; p < P; ++p) st.nb[s][p] = j >= 0 ? vdf + p * cs + (size_t)j * ld : st.own[p];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if constexpr (Stencil<D, T>::kLds) {
        st.lcf = lcf;
        st.ldd = ldd;
      } else if (lcf) {
        st.cf[s][d] = lcf[s * D + d];
        st.dd[s][d] = ldd[s * D + d];
      } else {
        st.cf[s][d] = j >= 0 ? (T)g.s_lsq[(size_t)(c * MAXF + s) * D + d] : (T)0;
        st.dd[s][d] = s < st.ns ? (T)g.s_d[(size_t)(c * MAXF + s) * D + d] : (T)0;
      }
    }
  }
}

// The stencil values of leaf k: the cell's own value and every neighbour's
// (a slot without an interior neighbour points at the cell's own row),
// loaded together so that they are in flight at once.
template <int D, typename T>
struct StencilVals {
  T phi[Cfg<D>::P];
  T nv[Cfg<D>::MAXF][Cfg<D>::P];
};

template <int D, typename T>
__device__ __forceinline__ void load_vals(const Stencil<D, T>& st, int k, StencilVals<D, T>& v) {
  constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF;
  const unsigned ko = (unsigned)k * (unsigned)sizeof(T);
#pragma unroll
  for (int p = 0; p < P; ++p) v.phi[p] = at_(st.own[p], ko);
#pragma unroll
  for (int s = 0; s < MAXF; ++s)
#pragma unroll
    for (int p = 0; p < P; ++p) v.nv[s][p] = at_(st.nb[s][p], ko);
}

// Least-squares gradient and Venkatakrishnan limiter at leaf k, in T.
// FULL: every one of the MAXF slots is a face with an interior neighbour
// (known at compile time, so the slot tests vanish from the leaf loop).
template <int D, typename T, bool FULL = false>
__device__ __forceinline__ void lim_parts(const Stencil<D, T>& st, const StencilVals<D, T>& sv, T (&phi)[Cfg<D>::P],
                                          T (&lim)[Cfg<D>::P], T (&grad)[Cfg<D>::P][D],
                                          T (&d2s)[Cfg<D>::P][Cfg<D>::MAXF]);

// Least-squares gradient, its increments grad . (x_f - x_i) towards the face
// midpoints (D2 of the limiter, d2s) and the Venkatakrishnan limiter L, per
// VDF component, in T.  FULL: every one of the MAXF slots is a face with an
// interior neighbour (known at compile time, so the slot tests vanish).
template <int D, typename T, bool FULL>
__device__ __forceinline__ void lim_parts(const Stencil<D, T>& st, const StencilVals<D, T>& sv, T (&phi)[Cfg<D>::P],
                                          T (&lim)[Cfg<D>::P], T (&grad)[Cfg<D>::P][D],
                                          T (&d2s)[Cfg<D>::P][Cfg<D>::MAXF]) {
  constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF;
  const int ns = FULL ? MAXF : st.ns;
  // the neighbour extrema are kept as differences from phi (rounding is
  // monotone, so max_j(v_j - phi) equals max_j(v_j) - phi exactly, and the
  // differences, being arithmetic results, need no NaN canonicalisation)
  T dmax[P], dmin[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    phi[p] = sv.phi[p];
    dmax[p] = 0;
    dmin[p] = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) grad[p][d] = 0;
  }
  const auto& nv = sv.nv;
#pragma unroll
  for (int s = 0; s < MAXF; ++s) {
    if (FULL || (st.nbmask & (1u << s))) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const T v = nv[s][p];
        const T dv = v - phi[p];
#pragma unroll
        for (int d = 0; d < D; ++d) grad[p][d] += dv * st.CF(s, d);
        dmax[p] = fmax(dv, dmax[p]);
        dmin[p] = fmin(dv, dmin[p]);
      }
    }
  }
  // Venkatakrishnan: psi_f = N/Dn with, for a = |D2| and b = |D1| (same sign),
  //   N = b^2 + eps^2 + 2ab,  Dn = b^2 + 2a^2 + ab + eps^2   (psi = 1 if D2 = 0),
  // which is the paper's expression divided through by D2.  a, b and eps are
  // scaled by the power of two just above the largest of them (exact), the
  // minimum over faces is kept as a fraction by cross-multiplication, and
  // one division ends it.
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const T up0 = dmax[p], dn0 = -dmin[p];
    T m = fmax(up0, dn0);
#pragma unroll
    for (int s = 0; s < MAXF; ++s) {
      T d2 = 0;
#pragma unroll
      for (int d = 0; d < D; ++d) d2 += grad[p][d] * st.DD(s, d);
      d2s[p][s] = d2;
      m = fmax(fabs(d2), m);
    }
    lim[p] = 1;
    // below the smallest normal number the stencil differences carry no
    // information (and the scale would overflow): leave the slope unlimited
    if ((FULL || ns > 0) && m > (sizeof(T) == 8 ? (T)1e-300 : (T)1e-36)) {
      int ex;
      (void)frexp(m, &ex);                             // m = f 2^ex, f in [0.5, 1)
      const T inv = ldexp((T)1, -ex);                  // scaled values lie in [0, 1)
      // eps^2 beyond this makes psi = 1 to working precision; the clamp keeps
      // the cross products below the overflow threshold of T.  The tiny term
      // keeps c > 0 where b and eps vanish (D2 = 0 gives a = 0 and N = Dn = c
      // exactly, psi = 1).
      const T e2 = fmin(st.eps2 * inv * inv, sizeof(T) == 8 ? (T)1e30 : (T)1e15) +
                   (sizeof(T) == 8 ? (T)1e-300 : (T)1e-30);
      const T up = up0 * inv, dn = dn0 * inv;
      T Nm = 1, Dm = 0;                                // running minimum, starts at +inf
#pragma unroll
      for (int s = 0; s < MAXF; ++s) {
        if (FULL || s < ns) {
          const T a = fabs(d2s[p][s]) * inv;
          const T b = d2s[p][s] > (T)0 ? up : dn;
          const T c = b * b + e2;
          const T a2 = a + a;
          const T Nn = a2 * b + c;
          const T Dd = a * (a2 + b) + c;
          if (FULL && s == 0) {
            Nm = Nn;
            Dm = Dd;
          } else if (Nn * Dm < Nm * Dd) {
            Nm = Nn;
            Dm = Dd;
          }
        }
      }
      // FP32: the hardware reciprocal (1 ulp) and one product in place of the
      // correctly rounded quotient; Dm lies in [1e-30, 1e16], a normal range
      if constexpr (sizeof(T) == 4)
        lim[p] = Nm * __builtin_amdgcn_rcpf(Dm);
      else
        lim[p] = Nm / Dm;
    }
  }
}

// ------------------------------------------------------------ pass A (S4)
// Per cell and leaf: limited gradient, and the upwind reconstruction at
// x_f - xi h for every face where this cell is upwind, stored to the
// interface buffer (exactly one writer per face and leaf), and the raw
// moments of those reconstructions over the workgroup's leaves (Eq.
// w_interface), one partial per (face, side, leaf chunk): the face's moments
// are the sum of its two sides' partials over the chunks, each leaf counted
// once (on its upwind side).  Grid (cells, leaf chunks) with cells fastest,
// so that a cell and its neighbours read the same chunk of their rows at
// about the same time.
//
// Raw moment slots (NM per face): m0, m1[D], m2[D(D+1)/2] (upper triangle,
// row by row), e = sum A (|xi|^2 G + H)/2, e1[D] = sum A xi (|xi|^2 G + H)/2.

// Threads of a pass-A workgroup: one wave per face slot, so that after the
// reconstruction of a block of NT leaves (one leaf per thread) wave s sums
// the moments of face s over the block (MAXF leaves per lane, from LDS).
template <int D>
constexpr int passA_threads() { return 64 * Cfg<D>::MAXF; }

// Sums of the face moments: FP64 in the FP64 form; in the FP32 form FP32
// lane sums of at most chunk/64 terms per face (a blocked sum whose rounding
// stays at the order of the FP32 storage's), added across lanes, workgroups
// and chunks in FP64.
template <typename T> struct MomAcc { using type = double; };
template <> struct MomAcc<float> { using type = float; };

template <int D, typename A>
__device__ __forceinline__ void face_mom_acc(A* m, A aw, A hw, const A (&x)[D], A G, A H) {
  A x2 = x[0] * x[0];
#pragma unroll
  for (int d = 1; d < D; ++d) x2 += x[d] * x[d];
  const A aG = aw * G;
  A ax[D];
#pragma unroll
  for (int d = 0; d < D; ++d) ax[d] = aG * x[d];
  int t = 0;
  m[t++] += aG;
#pragma unroll
  for (int d = 0; d < D; ++d) m[t++] += ax[d];
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int e = d; e < D; ++e) m[t++] += ax[d] * x[e];
  const A eh = hw * (x2 * G + H);
  m[t++] += eh;
#pragma unroll
  for (int d = 0; d < D; ++d) m[t++] += eh * x[d];
}

// LDS of one pass-A workgroup: the per-cell constants, and one block of
// reconstructions for the face sums: the upwind value of each face (0 where
// the cell is downwind), the leaf centre and weight.
template <int D, typename T>
struct PassAShared {
  static constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF, NT = passA_threads<D>();
  using A = typename MomAcc<T>::type;
  T cf[MAXF * D], dd[MAXF * D];
  double nrm[MAXF * D], sig[MAXF];
  A u[MAXF][P][NT];
  A x[D][NT];
  A a[NT];
};

template <int D, typename T, bool FULL>
__device__ __forceinline__ void passA_cell(PassAShared<D, T>& sh, const Geo& g, const Leaves& L,
                                           const T* __restrict__ vdf, const double* __restrict__ bcpair, double h,
                                           T* __restrict__ fv, double* __restrict__ fmom, int nchs, int i, int k0,
                                           int k1, int by) {
  constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF, NM = Cfg<D>::NM, NT = passA_threads<D>();
  using A = typename MomAcc<T>::type;
  T* const s_cf = sh.cf;
  T* const s_dd = sh.dd;
  double* const s_nrm = sh.nrm;
  double* const s_sig = sh.sig;
  auto& s_u = sh.u;
  auto& s_x = sh.x;
  auto& s_a = sh.a;
  const size_t cs = (size_t)g.nc * L.ld;
  const size_t fs = (size_t)g.nf * L.ld;   // component stride of the interface buffer
  // where the per-cell constants live: scalar registers (loaded from global
  // memory), vector registers (staged through LDS) or LDS itself.  In 2-D
  // the face normals go through LDS (fewer scalar spills), and in 2-D FP32
  // also the LSQ coefficients and face offsets.  3-D reads all of them from
  // LDS at their use, behind a compiler memory barrier per leaf, so they
  // occupy neither scalar nor vector registers across the leaf loop
  // (sphere FP32 pass A 38.7 -> 33.3 ms).
  constexpr bool lds_consts = (D == 2 && sizeof(T) == 4) || Stencil<D, T>::kLds;
  constexpr bool lds_nrm = D == 2 || Stencil<D, T>::kLds;
  Stencil<D, T> st;
  double nrm[MAXF][D];
  unsigned lside = 0;          // bit s: the cell is the L side of face s
  T* row[MAXF][P];
  if constexpr (lds_nrm) {
    const int ns = g.nslot[i];
    if (threadIdx.x < MAXF * D) {
      const int s = threadIdx.x / D, d = threadIdx.x % D;
      const int j = s < ns ? g.s_nbr[i * MAXF + s] : -1;
      const int f = s < ns ? g.s_face[i * MAXF + s] : 0;
      if constexpr (lds_consts) {
        s_cf[threadIdx.x] = j >= 0 ? (T)g.s_lsq[(size_t)i * MAXF * D + threadIdx.x] : (T)0;
        s_dd[threadIdx.x] = s < ns ? (T)g.s_d[(size_t)i * MAXF * D + threadIdx.x] : (T)0;
      }
      s_nrm[threadIdx.x] = g.f_nrm[(size_t)f * D + d];
      if (d == 0) s_sig[s] = s < ns ? g.s_sig[i * MAXF + s] : 0.0;
    }
    __syncthreads();
  }
  if constexpr (lds_consts) {
    load_stencil<D, T>(g, vdf, cs, L.ld, i, st, s_cf, s_dd);
  } else {
    load_stencil<D, T>(g, vdf, cs, L.ld, i, st);
  }
  const int ns = FULL ? MAXF : st.ns;
#pragma unroll
  for (int s = 0; s < MAXF; ++s) {
    const int f = (FULL || s < ns) ? g.s_face[i * MAXF + s] : 0;
    if constexpr (lds_nrm) {
      if (s_sig[s] > 0.0) lside |= 1u << s;
#pragma unroll
      for (int d = 0; d < D; ++d) nrm[s][d] = s_nrm[s * D + d];
    } else {
      if ((FULL || s < ns) && g.s_sig[i * MAXF + s] > 0.0) lside |= 1u << s;
#pragma unroll
      for (int d = 0; d < D; ++d) nrm[s][d] = g.f_nrm[(size_t)f * D + d];
    }
#pragma unroll
    for (int p = 0; p < P; ++p) row[s][p] = fv + p * fs + (size_t)f * L.ld;
  }
  // wave w sums face w: its moment accumulators (NM per lane)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  A acc[NM];
#pragma unroll
  for (int t = 0; t < NM; ++t) acc[t] = 0;
  const T th = (T)h;
  // the loads of the next block are issued before the face sums of this one,
  // so that they are in flight across the barriers
  StencilVals<D, T> sv;
  double xi_n[D], aw_n = 0.0;
  auto load_leaf = [&](int k) {
    load_vals<D, T>(st, k, sv);
#pragma unroll
    for (int d = 0; d < D; ++d) xi_n[d] = at_(L.xi + (size_t)d * L.cap, (unsigned)k * 8u);
    aw_n = at_(L.w, (unsigned)k * 8u);
  };
  if (k0 + (int)threadIdx.x < k1) load_leaf(k0 + threadIdx.x);
  for (int kb = k0; kb < k1; kb += NT) {
    const int k = kb + threadIdx.x;
    if (k < k1) {
      double xi[D];
#pragma unroll
      for (int d = 0; d < D; ++d) xi[d] = xi_n[d];
      const double aw_k = aw_n;
      T phi[P], lim[P], grad[P][D], d2s[P][MAXF];
      // re-read the LDS constants below instead of keeping them live
      if constexpr (Stencil<D, T>::kLds) __asm__ volatile("" ::: "memory");
      lim_parts<D, T, FULL>(st, sv, phi, lim, grad, d2s);
      // phibar = phi + L grad . (x_f - x_i) - h L grad . xi: the first product
      // is the limiter's D2 of the face, the second is shared by the faces
      T base[P];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        T gx = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) gx += grad[p][d] * (T)xi[d];
        base[p] = phi[p] - th * lim[p] * gx;
      }
#pragma unroll
      for (int s = 0; s < MAXF; ++s) {
        A u[P];
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = 0;
        if (FULL || s < ns) {
          const double sn = normal_speed<D>(xi, Stencil<D, T>::kLds ? s_nrm + s * D : nrm[s]);
          // L side: upwind for sn >= 0; R side: for sn < 0, the complement
          // (sn is finite).  One compare and a lane-mask xor with the
          // uniform side bit.
          const bool up = (sn >= 0.0) != !((lside >> s) & 1u);
          if (up) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
              const T v = base[p] + lim[p] * d2s[p][s];
              __builtin_nontemporal_store(v, ptr_at_(row[s][p], (unsigned)k * (unsigned)sizeof(T)));   // read by pass C only
              u[p] = (A)v;
            }
          } else if (!FULL && !((st.nbmask >> s) & 1u)) {
            // incoming leaf of a boundary face: the wall or far-field
            // Maxwellian, unscaled (the wall density ratio is applied in pass C)
            const int bc = -1 - g.f_R[g.s_face[i * MAXF + s]];
#pragma unroll
            for (int p = 0; p < P; ++p)
              __builtin_nontemporal_store((T)bcpair[((size_t)bc * P + p) * L.cap + k],
                                          ptr_at_(row[s][p], (unsigned)k * (unsigned)sizeof(T)));
          }
        }
#pragma unroll
        for (int p = 0; p < P; ++p) s_u[s][p][threadIdx.x] = u[p];
      }
#pragma unroll
      for (int d = 0; d < D; ++d) s_x[d][threadIdx.x] = (A)xi[d];
      s_a[threadIdx.x] = (A)aw_k;
      if (k + NT < k1) load_leaf(k + NT);
    } else {
#pragma unroll
      for (int s = 0; s < MAXF; ++s)
#pragma unroll
        for (int p = 0; p < P; ++p) s_u[s][p][threadIdx.x] = 0;
      s_a[threadIdx.x] = 0;
#pragma unroll
      for (int d = 0; d < D; ++d) s_x[d][threadIdx.x] = 0;
    }
    __syncthreads();
    // the face of this wave: moments of its upwind values over the block
    if (FULL || wave < ns) {
#pragma unroll
      for (int q = 0; q < NT / 64; ++q) {
        const int j = q * 64 + lane;
        A x[D];
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = s_x[d][j];
        const A aw = s_a[j];
        face_mom_acc<D, A>(acc, aw, (A)0.5 * aw, x, s_u[wave][0][j], P == 2 ? s_u[wave][P - 1][j] : (A)0);
      }
    }
    __syncthreads();
  }
  // one partial per (face, side, chunk): the wave's lanes added in FP64
  if (FULL || wave < ns) {
    double tot[NM];
#pragma unroll
    for (int t = 0; t < NM; ++t) {
      tot[t] = (double)acc[t];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) tot[t] += __shfl_xor(tot[t], o);
    }
    if (lane < NM) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < NM; ++t)
        if (t == lane) v = tot[t];
      const int f = g.s_face[i * MAXF + wave];
      const int side = g.s_sig[i * MAXF + wave] > 0.0 ? 0 : 1;
      fmom[(((size_t)f * 2 + side) * nchs + by) * NM + lane] = v;
    }
  }
}

template <int D, typename T>
__device__ __forceinline__ void d_passA(Geo g, Leaves L, const T* __restrict__ vdf, const double* __restrict__ bcpair,
                                        double h, T* __restrict__ fv, double* __restrict__ fmom, int nchs, int chunk,
                                        int bx, int by) {
  constexpr int MAXF = Cfg<D>::MAXF;
  const int i = xcd_cell(g, bx);
  if (i < 0) return;
  const int k0 = by * chunk, k1 = min(L.n, k0 + chunk);
  // a cell whose every slot is a face with an interior neighbour takes the
  // specialised loop (no slot tests); others (boundary cells, cells with
  // fewer faces) the general one
  bool full = g.nslot[i] == MAXF;
#pragma unroll
  for (int s = 0; s < MAXF; ++s) full = full && g.s_nbr[i * MAXF + s] >= 0;
  __shared__ PassAShared<D, T> sh;
  if (full)
    passA_cell<D, T, true>(sh, g, L, vdf, bcpair, h, fv, fmom, nchs, i, k0, k1, by);
  else
    passA_cell<D, T, false>(sh, g, L, vdf, bcpair, h, fv, fmom, nchs, i, k0, k1, by);
}

// Waves per SIMD pass A asks for: the face-moment accumulators (MAXF x NM
// lane sums) and the limiter's live values share the vector registers.
template <int D, typename T>
constexpr int passA_waves() { return D == 2 ? (sizeof(T) == 8 ? 3 : 5) : (sizeof(T) == 8 ? 3 : 4); }

template <int D, typename T>
__global__ __launch_bounds__(passA_threads<D>(), (passA_waves<D, T>())) void k_passA(Geo g, Leaves L, const T* __restrict__ vdf,
                                                                      const double* __restrict__ bcpair, double h,
                                                                      T* __restrict__ fv, double* __restrict__ fmom,
                                                                      int nchs, int chunk) {
  d_passA<D, T>(g, L, vdf, bcpair, h, fv, fmom, nchs, chunk, blockIdx.x, blockIdx.y);
}

// Flux of a raw-moment set through normal n: (n.m1, n.m2, n.e1).
template <int D>
__device__ __forceinline__ void raw_flux(const double* m, const double* n, double* F) {
  F[0] = 0.0;
  for (int d = 0; d < D; ++d) F[0] += n[d] * m[1 + d];
  int idx[3][3];
  int t = 1 + D;
  for (int d = 0; d < D; ++d)
    for (int e = d; e < D; ++e) { idx[d][e] = t; idx[e][d] = t; ++t; }
  for (int d = 0; d < D; ++d) {
    double v = 0.0;
    for (int e = 0; e < D; ++e) v += n[e] * m[idx[d][e]];
    F[1 + d] = v;
  }
  const int e1 = 2 + D + D * (D + 1) / 2;
  double v = 0.0;
  for (int d = 0; d < D; ++d) v += n[d] * m[e1 + d];
  F[D + 1] = v;
}

// ------------------------------------------------------ interface (S5-S8)
// d_face_eq: from the raw moments of the reconstructed VDF (Eq.
// w_interface; on a boundary face over the outgoing leaves only), summed
// from the partials pass A wrote: interior face: interface state, tau, heat
// flux relaxed over h at rate Pr/tau, Shakhov record and blend weights, then
// the flux F = a sum A s psi phibar + b sum A s psi g_f with g_f evaluated in
// R from the record.  Boundary face: outgoing flux plus the incoming wall
// (zero net mass flux, rho_w) or far-field Maxwellian flux.

// Faces per face_eq workgroup: each leaf is loaded once for all of them and
// their records are formed in parallel, one thread per face.
#ifndef AVS_FACE_BATCH2
#define AVS_FACE_BATCH2 4
#endif
#ifndef AVS_FACE_BATCH3
#define AVS_FACE_BATCH3 4
#endif
template <int D>
constexpr int face_batch() { return D == 2 ? AVS_FACE_BATCH2 : AVS_FACE_BATCH3; }

template <int D, typename R>
__device__ __forceinline__ void d_face_eq(Geo g, Leaves L, VGrid vg, GasP gas, double h, const double* __restrict__ bden,
                                          const double* __restrict__ bfin, const double* __restrict__ fmom, int nchs,
                                          int nch, double* __restrict__ fpar, double* __restrict__ F,
                                          int* __restrict__ bad, int bx) {
  constexpr int NM = Cfg<D>::NM, N = D + 2, FB = face_batch<D>();
  extern __shared__ double lds_d[];
  R* tab = reinterpret_cast<R*>(lds_d);       // FB tables of D x numax
  __shared__ double red[4 * FB * N];
  __shared__ double spar[FB][NPAR];
  __shared__ R rp[FB][NPAR];
  __shared__ double sF[FB][N];
  __shared__ double sm[FB][NM];
  __shared__ double snrm[FB][D];
  __shared__ int sok[FB];
  const int f0 = bx * FB;
  const int nfb = min(FB, g.nf - f0);
  // raw moments of each interface VDF: the partials of pass A, chunk by chunk,
  // L side then R side (a boundary face has its interior side only)
  if (threadIdx.x < FB * NM) {
    const int s = threadIdx.x / NM, t = threadIdx.x - s * NM;
    double v = 0.0;
    if (s < nfb) {
      const int f = f0 + s;
      const double* p0 = fmom + (size_t)f * 2 * nchs * NM + t;
      const double* p1 = p0 + (size_t)nchs * NM;
      const bool two = g.f_R[f] >= 0;
      for (int c = 0; c < nch; ++c) {
        v += p0[(size_t)c * NM];
        if (two) v += p1[(size_t)c * NM];
      }
    }
    sm[s][t] = v;
  }
  __syncthreads();
  // one thread per face: interface state, tau, relaxed heat flux, record and
  // blend weights (interior), or the boundary flux
  if (threadIdx.x < FB) {
    const int s = threadIdx.x;
    int ok = 0;
    if (s < nfb) {
      const int f = f0 + s;
      const int Rc = g.f_R[f];
      double n[D], m[NM];
      for (int d = 0; d < D; ++d) {
        n[d] = g.f_nrm[(size_t)f * D + d];
        snrm[s][d] = n[d];
      }
      for (int t = 0; t < NM; ++t) m[t] = sm[s][t];
      if (Rc >= 0) {
        const double rho = m[0];
        double U[D], ke = 0.0;
        for (int d = 0; d < D; ++d) { U[d] = m[1 + d] / rho; ke += U[d] * U[d]; }
        const int ie = 1 + D + D * (D + 1) / 2;
        const double E = m[ie];
        const double T = (E - 0.5 * rho * ke) / (1.5 * rho * gas.R);
        if (!(rho > 0.0 && T > 0.0)) {
          atomicMin(bad, g.nc + f);
        } else {
          // q about U from raw moments: e1_d - U_d E - sum_e U_e (m2_de - rho U_d U_e) + |U|^2/2 (m1_d - U_d rho)
          int idx[3][3];
          int t = 1 + D;
          for (int d = 0; d < D; ++d)
            for (int e = d; e < D; ++e) { idx[d][e] = t; idx[e][d] = t; ++t; }
          double q[D];
          for (int d = 0; d < D; ++d) {
            double v = m[ie + 1 + d] - U[d] * E;
            for (int e = 0; e < D; ++e) v -= U[e] * (m[idx[d][e]] - rho * U[d] * U[e]);
            v += 0.5 * ke * (m[1 + d] - U[d] * rho);
            q[d] = v;
          }
          const double tf = tau_of(rho, T, gas);
          const double qs = tf / (tf + h * gas.Pr);
          for (int d = 0; d < D; ++d) q[d] *= qs;
          eq_record<D>(spar[s], rho, U, T, q, gas);
          spar[s][P_A] = tf / (tf + h);
          spar[s][P_B] = h / (tf + h);
          raw_flux<D>(m, n, sF[s]);
          ok = 1;
        }
      } else {
        const int bc = -1 - Rc;
        double Fo[N];
        raw_flux<D>(m, n, Fo);
        const double* fin = bfin + (size_t)f * N;
        double scale = 1.0;
        if (g.bc_kind[bc] == 0) {
          scale = Fo[0] / bden[f];
          fpar[(size_t)f * NPAR] = scale;
        }
        for (int t = 0; t < N; ++t) F[(size_t)f * N + t] = Fo[t] + scale * fin[t];
      }
    }
    sok[s] = ok;
  }
  __syncthreads();
  int any = 0;
#pragma unroll
  for (int s = 0; s < FB; ++s) any |= sok[s];
  if (!any) return;
  for (int t = threadIdx.x; t < FB * NPAR; t += BLOCK) {
    const int s = t / NPAR, m = t - s * NPAR;
    if (sok[s]) {
      fpar[(size_t)(f0 + s) * NPAR + m] = spar[s][m];
      rp[s][m] = (R)spar[s][m];
    }
  }
#pragma unroll
  for (int s = 0; s < FB; ++s)
    if (sok[s]) build_tab_r<D, R>(tab + s * D * vg.numax, spar[s], vg);
  __syncthreads();
  double acc[FB * N];
#pragma unroll
  for (int t = 0; t < FB * N; ++t) acc[t] = 0.0;
  // 2-D: the next leaf's entry is loaded while this one is used (in 3-D the
  // registers it takes would cost a wave per SIMD)
  constexpr bool PRE = D == 2;
  double xi_n[D], A_n = 0.0;
  int u_n[D];
  if (PRE && (int)threadIdx.x < L.n) leaf_load_rows<D>(L, threadIdx.x, xi_n, A_n, u_n);
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    if constexpr (PRE) {
      A = A_n;
#pragma unroll
      for (int d = 0; d < D; ++d) { xi[d] = xi_n[d]; u[d] = u_n[d]; }
      if (k + BLOCK < L.n) leaf_load_rows<D>(L, k + BLOCK, xi_n, A_n, u_n);
    } else {
      leaf_load_rows<D>(L, k, xi, A, u);
    }
    R xr[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xr[d] = (R)xi[d];
    double xi2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) xi2 += xi[d] * xi[d];
#pragma unroll
    for (int s = 0; s < FB; ++s) {
      if (!sok[s]) continue;
      const R gv = maxw_r<D, R>(rp[s], tab + s * D * vg.numax, vg.numax, u);
      R G, H;
      shakhov_r<D, R>(rp[s], gv, xr, G, H);
      const double sn = flux_weight<D>(xi, snrm[s]);
      mom_acc<D>(acc + s * N, A * sn, xi, xi2, (double)G, (double)H);
    }
  }
  block_sum<FB * N>(acc, red);
  // static indices into acc (a dynamic one would move it to scratch memory)
#pragma unroll
  for (int s = 0; s < FB; ++s) {
    if (threadIdx.x == s && sok[s]) {
      const double a = spar[s][P_A], b = spar[s][P_B];
#pragma unroll
      for (int t = 0; t < N; ++t) F[(size_t)(f0 + s) * N + t] = a * sF[s][t] + b * acc[s * N + t];
    }
  }
}

template <int D, typename R>
__global__ __launch_bounds__(BLOCK) void k_face_eq(Geo g, Leaves L, VGrid vg, GasP gas, double h,
                                                  const double* __restrict__ bden, const double* __restrict__ bfin,
                                                  const double* __restrict__ fmom, int nchs, int nch,
                                                  double* __restrict__ fpar, double* __restrict__ F,
                                                  int* __restrict__ bad) {
  d_face_eq<D, R>(g, L, vg, gas, h, bden, bfin, fmom, nchs, nch, fpar, F, bad, blockIdx.x);
}


// ------------------------------------------------------ macro update (S8-S9)
// Cell record of the relaxation target from the new state w of cell i:
// Shakhov parameters with q^n, dt/tau, rho and T.
template <int D>
__device__ __forceinline__ void target_record(int i, const double* w, const GasP& gas, double dt,
                                              const double* __restrict__ qcur, double* __restrict__ tpar,
                                              int* __restrict__ bad) {
  double rho, U[D], T;
  if (!prim_from_W<D>(w, gas, rho, U, T)) { atomicMin(bad, i); rho = 1.0; T = 1.0; }
  double* par = tpar + (size_t)i * NPAR;
  eq_record<D>(par, rho, U, T, qcur + (size_t)i * D, gas);
  par[P_A] = dt / tau_of(rho, T, gas);
  par[P_RHO] = rho;
  par[P_T] = T;
}

template <int D>
__device__ __forceinline__ void d_macro(Geo g, GasP gas, double dt, const double* __restrict__ F, const double* __restrict__ W,
                        double* __restrict__ Wn, const double* __restrict__ qcur, double* __restrict__ tpar,
                        int* __restrict__ bad, int bx, int by) {
  constexpr int MAXF = Cfg<D>::MAXF, N = D + 2;
  const int i = bx * BLOCK + threadIdx.x;
  if (i >= g.nc) return;
  const int ns = g.nslot[i];
  double Fs[N];
  for (int m = 0; m < N; ++m) Fs[m] = 0.0;
  for (int s = 0; s < ns; ++s) {
    const int f = g.s_face[i * MAXF + s];
    const double sa = g.s_sigA[i * MAXF + s];
    for (int m = 0; m < N; ++m) Fs[m] += sa * F[(size_t)f * N + m];
  }
  double w[N];
  const double dtv = g.dtv[i];
  for (int m = 0; m < N; ++m) {
    w[m] = W[(size_t)i * N + m] - dtv * Fs[m];
    Wn[(size_t)i * N + m] = w[m];
  }
  target_record<D>(i, w, gas, dt, qcur, tpar, bad);
}

template <int D>
__global__ void k_macro(Geo g, GasP gas, double dt, const double* __restrict__ F, const double* __restrict__ W,
                        double* __restrict__ Wn, const double* __restrict__ qcur, double* __restrict__ tpar,
                        int* __restrict__ bad) {
  d_macro<D>(g, gas, dt, F, W, Wn, qcur, tpar, bad, blockIdx.x, blockIdx.y);
}

// --------------------------------------- conservative relaxation target (S9)
// lambda such that closure(Shakhov(W^{n+1}, q^n)) has moments W^{n+1}; the
// Shakhov values are evaluated in R, the moment and Gram sums in FP64 and
// the (D+2)x(D+2) solve in FP64.
template <int D, typename R>
__device__ __forceinline__ void d_target(Geo g, Leaves L, VGrid vg, const double* __restrict__ tpar,
                                                   const double* __restrict__ Wn, double* __restrict__ lam,
                                                   int* __restrict__ bad, int bx, int by) {
  constexpr int N = D + 2, NS = Cfg<D>::NS;
  extern __shared__ double lds_d[];
  R* tab = reinterpret_cast<R*>(lds_d);
  __shared__ double red[4 * (N + NS)];
  __shared__ R rp[NPAR];
  __shared__ ClosureWork<D> cw;
  const int i = bx;
  const double* par = tpar + (size_t)i * NPAR;
  if (threadIdx.x < NPAR) rp[threadIdx.x] = (R)par[threadIdx.x];
  build_tab_r<D, R>(tab, par, vg);
  __syncthreads();
  double acc[N + NS];
#pragma unroll
  for (int m = 0; m < N + NS; ++m) acc[m] = 0.0;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    leaf_load_rows<D>(L, k, xi, A, u);
    R xr[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xr[d] = (R)xi[d];
    const R gr = maxw_r<D, R>(rp, tab, vg.numax, u);
    R Gr, Hr;
    shakhov_r<D, R>(rp, gr, xr, Gr, Hr);
    const double gv = gr;
    double c[D], c2 = 0.0, xi2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) { c[d] = xi[d] - par[P_U + d]; c2 += c[d] * c[d]; xi2 += xi[d] * xi[d]; }
    mom_acc<D>(acc, A, xi, xi2, (double)Gr, (double)Hr);
    gram_acc<D>(acc + N, A * gv, c, c2);
  }
  block_sum<N + NS>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < NS; ++m) cw.S[m] = acc[N + m];
    gram_to_J<D>(cw.S, par, cw.J);
#pragma unroll
    for (int m = 0; m < N; ++m) cw.b[m] = Wn[(size_t)i * N + m] - acc[m];
    if (!solve_small<N>(cw.J, cw.b, cw.x)) { atomicMin(bad, i); for (int m = 0; m < N; ++m) cw.x[m] = 0.0; }
    for (int m = 0; m < N; ++m) lam[(size_t)i * N + m] = cw.x[m];
  }
}

template <int D, typename R>
__global__ __launch_bounds__(BLOCK) void k_target(Geo g, Leaves L, VGrid vg, const double* __restrict__ tpar,
                                                   const double* __restrict__ Wn, double* __restrict__ lam,
                                                   int* __restrict__ bad) {
  d_target<D, R>(g, L, vg, tpar, Wn, lam, bad, blockIdx.x, blockIdx.y);
}

// -------------------------------------------------- pass C (S6, S7, S10)
// Interface VDFs of every face of the cell (upwind reconstruction from the
// interface buffer, blended with the interface Shakhov equilibrium; on
// incoming leaves of a boundary face the wall or far-field Maxwellian that
// pass A stored there, times the wall density ratio), flux divergence,
// relaxation towards the closed Shakhov target, store phi^{n+1}, and the
// moments and heat flux of phi^{n+1} for the next step.  Arithmetic in T,
// sums in FP64; the upwind sign in FP64 in both forms.
//
// All loads of a leaf (leaf table, phi, every interface row) are issued
// before any of them is used.  In 2-D FP64 the loads of leaf k + BLOCK are
// also issued before leaf k is processed (two register sets used in turn),
// so that a wave keeps two leaves of memory traffic in flight; the other
// forms have fewer spare registers and run faster with one.
template <int D, typename T>
constexpr bool passc_two_leaves() { return D == 2 && sizeof(T) == 8; }

template <int D, typename T>
struct LeafIn {
  static constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF;
  double xi[D], A;
  int u[D];
  T phi[P];
  T row[MAXF][P];
};

// With RES set, the kernel stores the explicit increment of the implicit
// micro system instead, (dt/tau~)(g~ - phi^n) - (dt/V) sum_f sigma A xi.n
// phi_f (Eq. SGS_phi's right-hand side times dt/V), and skips the moments.
template <int D, typename T, bool RES = false, bool TWO = passc_two_leaves<D, T>()>
__device__ __forceinline__ void d_passC(Geo g, Leaves L, VGrid vg, const T* __restrict__ vin,
                                        const T* __restrict__ fv, T* __restrict__ vout,
                                        const double* __restrict__ fpar, const double* __restrict__ tpar,
                                        const double* __restrict__ lam, double* __restrict__ mom,
                                        double* __restrict__ qout, int bx) {
  constexpr int P = Cfg<D>::P, MAXF = Cfg<D>::MAXF, N = D + 2;
  extern __shared__ double lds_d[];
  T* lds = reinterpret_cast<T*>(lds_d);
  __shared__ double red[4 * (N + D)];
  __shared__ T spar[(MAXF + 1) * NPAR];
  __shared__ double snrm[MAXF][D];
  __shared__ T snrt[MAXF][D];
  __shared__ int sface[MAXF], snbr[MAXF];
  __shared__ T ssa[MAXF], ssc[MAXF];
  __shared__ T slam[N];
  const int i = xcd_cell(g, bx);
  if (i < 0) return;
  const int ns = g.nslot[i];
  const int nu = vg.numax;
  const size_t cs = (size_t)g.nc * L.ld;
  const size_t fs = (size_t)g.nf * L.ld;
  for (int t = threadIdx.x; t < (MAXF + 1) * NPAR; t += BLOCK) {
    const int s = t / NPAR, m = t - s * NPAR;
    double v = 0.0;
    if (s < MAXF) {
      if (s < ns) v = fpar[(size_t)g.s_face[i * MAXF + s] * NPAR + m];
    } else {
      v = tpar[(size_t)i * NPAR + m];
    }
    spar[t] = (T)v;
  }
  if (threadIdx.x < MAXF) {
    const int s = threadIdx.x;
    const int f = s < ns ? g.s_face[i * MAXF + s] : 0;
    sface[s] = f;
    snbr[s] = s < ns ? g.s_nbr[i * MAXF + s] : -1;
    ssa[s] = s < ns ? (T)g.s_sigA[i * MAXF + s] : (T)0;
    // wall: density ratio of the incoming Maxwellian (first record slot of a
    // boundary face); far field and interior faces: 1
    const bool wall = s < ns && g.f_R[f] < 0 && g.bc_kind[-1 - g.f_R[f]] == 0;
    ssc[s] = wall ? (T)fpar[(size_t)f * NPAR] : (T)1;
    for (int d = 0; d < D; ++d) {
      snrm[s][d] = g.f_nrm[(size_t)f * D + d];
      snrt[s][d] = (T)snrm[s][d];
    }
  }
  if (threadIdx.x < N) slam[threadIdx.x] = (T)lam[(size_t)i * N + threadIdx.x];
  // row pointers from global memory (scalar registers), so that every load
  // and store of the leaf loop is a scalar base plus one 32-bit lane offset
  const T* frow[MAXF][P];
  const T* vrow[P];
  T* orow[P];
#pragma unroll
  for (int s = 0; s < MAXF; ++s) {
    const size_t f = s < ns ? (size_t)g.s_face[i * MAXF + s] : 0;
#pragma unroll
    for (int p = 0; p < P; ++p) frow[s][p] = fv + p * fs + f * L.ld;
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    vrow[p] = vin + p * cs + (size_t)i * L.ld;
    orow[p] = vout + p * cs + (size_t)i * L.ld;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < MAXF; ++s) {
    if (s < ns && snbr[s] >= 0) build_tab_r<D, T>(lds + s * D * nu, fpar + (size_t)sface[s] * NPAR, vg);
  }
  build_tab_r<D, T>(lds + MAXF * D * nu, tpar + (size_t)i * NPAR, vg);
  __syncthreads();
  const T* tp = spar + MAXF * NPAR;
  // the unrolled face loop in 3-D and FP32 (2-D FP64, bound by HBM, is no
  // faster with it and fetches more)
  bool full = (D == 3 || sizeof(T) == 4) && ns == MAXF;
#pragma unroll
  for (int q = 0; q < MAXF; ++q) full = full && snbr[q] >= 0;
  const T dtt = tp[P_A], dtv = (T)g.dtv[i];
  const T inv = (T)1 / ((T)1 + dtt);
  double acc[N + D];
#pragma unroll
  for (int m = 0; m < N + D; ++m) acc[m] = 0.0;

  auto load = [&](int k, LeafIn<D, T>& x) {
    const unsigned ko = (unsigned)k * (unsigned)sizeof(T);
    leaf_load<D>(L, k, x.xi, x.A, x.u);
#pragma unroll
    for (int p = 0; p < P; ++p) x.phi[p] = at_(vrow[p], ko);
    // unconditional, so that all rows of the leaf are in flight together (a
    // slot beyond the cell's faces reads face 0 and is never used)
#pragma unroll
    for (int s = 0; s < MAXF; ++s)
#pragma unroll
      for (int p = 0; p < P; ++p) x.row[s][p] = at_(frow[s][p], ko);
  };
  auto process = [&](int k, const LeafIn<D, T>& x) {
    T xr[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xr[d] = (T)x.xi[d];
    T div[P];
#pragma unroll
    for (int p = 0; p < P; ++p) div[p] = 0;
    if (full) {
      // every slot an interior face: the face loop unrolled, rows taken by
      // static index.  The empty asm with a memory clobber makes each face
      // read its record from LDS where it is used; without it the compiler
      // keeps all the faces' records live across the leaf loop (168-256
      // VGPRs).
#pragma unroll
      for (int s = 0; s < MAXF; ++s) {
        __asm__ volatile("" ::: "memory");
        T pf[P];
#pragma unroll
        for (int p = 0; p < P; ++p) pf[p] = x.row[s][p];
        const T* par = spar + s * NPAR;
        const T gv = maxw_r<D, T>(par, lds + s * D * nu, nu, x.u);
        T G, H;
        shakhov_r<D, T>(par, gv, xr, G, H);
        pf[0] = par[P_A] * pf[0] + par[P_B] * G;
        if (P == 2) pf[P - 1] = par[P_A] * pf[P - 1] + par[P_B] * H;
        T sw;
        if constexpr (sizeof(T) == 8) {
          sw = normal_speed<D>(x.xi, snrm[s]);
        } else {
          sw = xr[0] * snrt[s][0];
#pragma unroll
          for (int d = 1; d < D; ++d) sw += xr[d] * snrt[s][d];
        }
        const T w = ssa[s] * sw;
#pragma unroll
        for (int p = 0; p < P; ++p) div[p] += w * pf[p];
      }
    } else
    // one face at a time: its record is read from LDS inside the loop, so
    // only one face's parameters are live in registers
#pragma unroll 1
    for (int s = 0; s < ns; ++s) {
      // static indices only (a dynamic index would move the rows to scratch memory)
      T pf[P];
#pragma unroll
      for (int q = 0; q < MAXF; ++q)
#pragma unroll
        for (int p = 0; p < P; ++p) pf[p] = q == s ? x.row[q][p] : (q == 0 ? (T)0 : pf[p]);
      T sw;     // xi . n, the flux weight
      if (snbr[s] >= 0) {
        const T* par = spar + s * NPAR;
        const T gv = maxw_r<D, T>(par, lds + s * D * nu, nu, x.u);
        T G, H;
        shakhov_r<D, T>(par, gv, xr, G, H);
        pf[0] = par[P_A] * pf[0] + par[P_B] * G;
        if (P == 2) pf[P - 1] = par[P_A] * pf[P - 1] + par[P_B] * H;
        // no side is chosen here, so the weight is formed in T (both cells
        // of the face form the same value: the flux stays antisymmetric)
        if constexpr (sizeof(T) == 8) {
          sw = normal_speed<D>(x.xi, snrm[s]);
        } else {
          sw = xr[0] * snrt[s][0];
#pragma unroll
          for (int d = 1; d < D; ++d) sw += xr[d] * snrt[s][d];
        }
      } else {
        // boundary face: the incoming side is taken in FP64, as in pass A
        const double sn = normal_speed<D>(x.xi, snrm[s]);
        if (sn < 0.0) {
#pragma unroll
          for (int p = 0; p < P; ++p) pf[p] = ssc[s] * pf[p];
        }
        sw = (T)sn;
      }
      const T w = ssa[s] * sw;
#pragma unroll
      for (int p = 0; p < P; ++p) div[p] += w * pf[p];
    }
    // closed Shakhov target
    const T gv = maxw_r<D, T>(tp, lds + MAXF * D * nu, nu, x.u);
    T G, H;
    shakhov_r<D, T>(tp, gv, xr, G, H);
    T c[D], c2 = 0, poly = slam[0];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      c[d] = xr[d] - tp[P_U + d];
      c2 += c[d] * c[d];
      poly += slam[1 + d] * c[d];
    }
    poly += slam[D + 1] * c2;
    const T tgt[2] = {G + poly * gv, H + poly * tp[P_RT] * gv};
    if constexpr (RES) {
#pragma unroll
      for (int p = 0; p < P; ++p)
        *ptr_at_(orow[p], (unsigned)k * (unsigned)sizeof(T)) = dtt * (tgt[p] - x.phi[p]) - dtv * div[p];
      return;
    }
    double nv[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const T st = (x.phi[p] + dtt * tgt[p] - dtv * div[p]) * inv;
      *ptr_at_(orow[p], (unsigned)k * (unsigned)sizeof(T)) = st;
      nv[p] = (double)st;
    }
    double xi2 = 0.0, cd[D], c2d = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      xi2 += x.xi[d] * x.xi[d];
      cd[d] = x.xi[d] - (double)tp[P_U + d];
      c2d += cd[d] * cd[d];
    }
    const double Hn = (P == 2) ? nv[P - 1] : 0.0;
    mom_acc<D>(acc, x.A, x.xi, xi2, nv[0], Hn);
    const double e = 0.5 * x.A * (c2d * nv[0] + Hn);
#pragma unroll
    for (int d = 0; d < D; ++d) acc[N + d] += e * cd[d];
  };

  if constexpr (!TWO) {
    for (int k = threadIdx.x; k < L.n; k += BLOCK) {
      LeafIn<D, T> x;
      load(k, x);
      process(k, x);
    }
  } else {
    LeafIn<D, T> x0, x1;
    int k = threadIdx.x;
    if (k < L.n) load(k, x0);
    for (; k < L.n; k += 2 * BLOCK) {
      if (k + BLOCK < L.n) load(k + BLOCK, x1);
      process(k, x0);
      if (k + BLOCK >= L.n) break;
      if (k + 2 * BLOCK < L.n) load(k + 2 * BLOCK, x0);
      process(k + BLOCK, x1);
    }
  }
  if constexpr (RES) return;
  block_sum<N + D>(acc, red);
  if (threadIdx.x == 0) {
    for (int m = 0; m < N; ++m) mom[(size_t)i * N + m] = acc[m];
    for (int d = 0; d < D; ++d) qout[(size_t)i * D + d] = acc[N + d];
  }
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK, (waves_hint<D, T>())) void k_passC(Geo g, Leaves L, VGrid vg, const T* __restrict__ vin,
                                                     const T* __restrict__ fv, T* __restrict__ vout,
                                                     const double* __restrict__ fpar, const double* __restrict__ tpar,
                                                     const double* __restrict__ lam, double* __restrict__ mom,
                                                     double* __restrict__ qout) {
  d_passC<D, T>(g, L, vg, vin, fv, vout, fpar, tpar, lam, mom, qout, blockIdx.x);
}

// ----------------------------------------------- boundary Maxwellians (S7)
// Per bc and leaf: the incoming Maxwellian pair (unit density for walls).
template <int D>
__device__ __forceinline__ void d_bc_pairs(Leaves L, GasP gas, int nbc, const int* __restrict__ kind,
                                           const double* __restrict__ prim, double* __restrict__ pair, int bx,
                                           int by) {
  constexpr int P = Cfg<D>::P;
  const int k = bx * BLOCK + threadIdx.x;
  const int b = by;
  if (k >= L.n) return;
  const double* st = prim + (size_t)b * (D + 2);
  const double rho = kind[b] == 0 ? 1.0 : st[0];
  const double T = st[1 + D], RT = gas.R * T;
  double c2 = 0.0;
  for (int d = 0; d < D; ++d) {
    const double c = L.xi[d * L.cap + k] - st[1 + d];
    c2 += c * c;
  }
  const double gv = rho * pow(2.0 * M_PI * RT, -0.5 * D) * exp(-c2 / (2.0 * RT));
  pair[((size_t)b * P + 0) * L.cap + k] = gv;
  if (P == 2) pair[((size_t)b * P + 1) * L.cap + k] = RT * gv;
}

template <int D>
__global__ void k_bc_pairs(Leaves L, GasP gas, int nbc, const int* __restrict__ kind, const double* __restrict__ prim,
                           double* __restrict__ pair) {
  d_bc_pairs<D>(L, gas, nbc, kind, prim, pair, blockIdx.x, blockIdx.y);
}

// Per boundary face: den = sum_{s<0} A |s| g_wall and Fin = sum_{s<0} A s psi pair.
template <int D>
__device__ __forceinline__ void d_bnd_tables(Geo g, Leaves L, const double* __restrict__ pair,
                                             double* __restrict__ bden, double* __restrict__ bfin, int bx) {
  constexpr int P = Cfg<D>::P, N = D + 2;
  __shared__ double red[4 * (N + 1)];
  const int f = g.f_bnd[bx];
  const int bc = -1 - g.f_R[f];
  double n[D];
  for (int d = 0; d < D; ++d) n[d] = g.f_nrm[(size_t)f * D + d];
  double acc[N + 1];
  for (int m = 0; m < N + 1; ++m) acc[m] = 0.0;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    leaf_load<D>(L, k, xi, A, u);
    const double sn = normal_speed<D>(xi, n);
    double xi2 = 0.0;
    for (int d = 0; d < D; ++d) xi2 += xi[d] * xi[d];
    if (sn < 0.0) {
      const double G = pair[((size_t)bc * P) * L.cap + k];
      const double H = P == 2 ? pair[((size_t)bc * P + 1) * L.cap + k] : 0.0;
      mom_acc<D>(acc, A * sn, xi, xi2, G, H);
      acc[N] += A * (-sn) * G;
    }
  }
  block_sum<N + 1>(acc, red);
  if (threadIdx.x == 0) {
    for (int m = 0; m < N; ++m) bfin[(size_t)f * N + m] = acc[m];
    bden[f] = acc[N];
  }
}

template <int D>
__global__ __launch_bounds__(BLOCK) void k_bnd_tables(Geo g, Leaves L, const double* __restrict__ pair,
                             double* __restrict__ bden, double* __restrict__ bfin) {
  d_bnd_tables<D>(g, L, pair, bden, bfin, blockIdx.x);
}

// ----------------------------------------------------- criterion (Sec. 3.4)
// Per-cell constants of the criterion, same operation order as the oracle.
template <int D>
__global__ void k_crit_cells(int nc, const double* __restrict__ W, double* __restrict__ cc) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
  const double* w = W + (size_t)i * (D + 2);
  const double rho = w[0];
  double U[D];
  for (int d = 0; d < D; ++d) U[d] = w[1 + d] / rho;
  double ke = U[0] * U[0];
  for (int d = 1; d < D; ++d) ke = ke + U[d] * U[d];
  const double eint = w[1 + D] - 0.5 * rho * ke;
  double* o = cc + (size_t)i * (D + 2);
  o[0] = rho;
  for (int d = 0; d < D; ++d) o[1 + d] = U[d];
  o[1 + D] = eint;
}

template <int D>
__device__ __forceinline__ double crit_one(const double (&xi)[D], double A, double G, double H, const double* cc) {
#pragma clang fp contract(off)
  double c = xi[0] - cc[1];
  double c2 = c * c;
  for (int d = 1; d < D; ++d) {
    c = xi[d] - cc[1 + d];
    c2 = c2 + c * c;
  }
  const double M1 = (A * G) / cc[0];
  const double M2 = (0.5 * (A * (c2 * G + H))) / cc[1 + D];
  return fmax(M1, M2);
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void k_crit_partial(Leaves L, int nc, const T* __restrict__ vdf,
                                                         const double* __restrict__ cc, double* __restrict__ part) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  const int grp = blockIdx.y;
  if (k >= L.n) return;
  const size_t cs = (size_t)nc * L.ld;
  double xi[D], A;
  int u[D];
  leaf_load<D>(L, k, xi, A, u);
  double m = -INFINITY;
  const int i1 = min(nc, (grp + 1) * CRIT_CELLS);
  for (int i = grp * CRIT_CELLS; i < i1; ++i) {
    const double G = ld_(vdf + (size_t)i * L.ld + k);
    const double H = D == 2 ? ld_(vdf + cs + (size_t)i * L.ld + k) : 0.0;
    m = fmax(m, crit_one<D>(xi, A, G, H, cc + (size_t)i * (D + 2)));
  }
  part[(size_t)grp * L.cap + k] = m;
}

// Max over cell groups and probe states; raw split/merge flags.
template <int D>
__global__ void k_crit_reduce(Leaves L, int ngrp, const double* __restrict__ part, int nprobe,
                              const double* __restrict__ probe_cc, const double* __restrict__ probe_prim, GasP gas,
                              double C1, double C2, int lmax, double* __restrict__ Mk, int8_t* __restrict__ raw) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= L.n) return;
  double m = -INFINITY;
  for (int t = 0; t < ngrp; ++t) m = fmax(m, part[(size_t)t * L.cap + k]);
  double xi[D], A;
  int u[D];
  leaf_load<D>(L, k, xi, A, u);
  for (int p = 0; p < nprobe; ++p) {
    const double* pr = probe_prim + (size_t)p * (D + 2);
    // the discrete Maxwellian pair in the oracle's association (exp and pow
    // are this library's: probe values agree to rounding, flags away from ties)
    const double rho = pr[0], T = pr[1 + D], R = gas.R;
    double c = xi[0] - pr[1];
    double c2 = c * c;
    for (int d = 1; d < D; ++d) {
      c = xi[d] - pr[1 + d];
      c2 = c2 + c * c;
    }
    const double gv = rho * pow(2.0 * M_PI * R * T, -0.5 * D) * exp(-c2 / (2.0 * R * T));
    m = fmax(m, crit_one<D>(xi, A, gv, D == 2 ? (double)(3 - D) * R * T * gv : 0.0, probe_cc + (size_t)p * (D + 2)));
  }
  Mk[k] = m;
  const int l = L.level[k];
  int8_t r = 0;
  if (m > C1 && l < lmax) r = 1;
  if (m < C2 && l > 0) r = -1;
  raw[k] = r;
}

// Separated-zone floor (Sec. 3.5) on the raw flags: an element centred in
// the open annulus lo2 < |xi|^2 < hi2 about the origin keeps at least level
// S.  A leaf there below S splits (below lmax); a merge candidate whose
// parent would be centred there below S is kept.  |xi|^2 is summed axis by
// axis, the parent's centre taken as the leaf geometry takes a centre.
template <int D>
__global__ void k_sep_floor(Leaves L, int lmax, int b0, int b1, int b2, double lo0, double lo1, double lo2,
                            double hi0, double hi1, double hi2, double r2lo, double r2hi, int S,
                            int8_t* __restrict__ raw) {
#pragma clang fp contract(off)
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= L.n) return;
  const int base[3] = {b0, b1, b2};
  const double lo[3] = {lo0, lo1, lo2}, hi[3] = {hi0, hi1, hi2};
  const int l = L.level[k];
  int8_t r = raw[k];
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double x = L.xi[d * L.cap + k];
    s = s + x * x;
  }
  if (r2lo < s && s < r2hi && l < S && l < lmax) r = 1;
  if (r == -1 && l > 0 && l - 1 < S) {
    s = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double h = (hi[d] - lo[d]) / (double)(base[d] << (l - 1));
      const double c = lo[d] + ((double)(L.idx[d * L.cap + k] >> 1) + 0.5) * h;
      s = s + c * c;
    }
    if (r2lo < s && s < r2hi) r = 0;
  }
  raw[k] = r;
}

// Effective flags (a brother group merges only if complete and unanimous)
// and the number of new leaves each old leaf produces.
template <int D>
__global__ void k_resolve(Leaves L, const int8_t* __restrict__ raw, int8_t* __restrict__ eff, int* __restrict__ cnt) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= L.n) return;
  const int8_t r = raw[k];
  const int l = L.level[k];
  int cnum = 0;
  for (int d = 0; d < D; ++d) cnum |= (L.idx[d * L.cap + k] & 1) << d;
  int8_t e = r;
  if (r == -1) {
    const int first = k - cnum;
    bool ok = first >= 0 && first + (1 << D) <= L.n;
    for (int c = 0; ok && c < (1 << D); ++c) {
      const int m = first + c;
      if (raw[m] != -1 || L.level[m] != l) { ok = false; break; }
      int cm = 0;
      for (int d = 0; d < D; ++d) {
        const int a = L.idx[d * L.cap + m], b = L.idx[d * L.cap + k];
        if ((a >> 1) != (b >> 1)) ok = false;
        cm |= (a & 1) << d;
      }
      if (cm != c) ok = false;
    }
    e = ok ? -1 : 0;
  }
  eff[k] = e;
  cnt[k] = e == 0 ? 1 : (e == 1 ? (1 << D) : (cnum == 0 ? 1 : 0));
}

// Exclusive scan of n counts in one workgroup (deterministic, any n).
__global__ __launch_bounds__(BLOCK) void k_scan(int n, const int* __restrict__ cnt, int* __restrict__ off) {
  __shared__ int part[BLOCK];
  const int per = (n + BLOCK - 1) / BLOCK;
  const int b = threadIdx.x * per, e = min(n, b + per);
  int s = 0;
  for (int k = b; k < e; ++k) s += cnt[k];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < BLOCK; ++t) { const int v = part[t]; part[t] = run; run += v; }
    off[n] = run;
  }
  __syncthreads();
  int run = part[threadIdx.x];
  for (int k = b; k < e; ++k) { off[k] = run; run += cnt[k]; }
}

template <int D>
__global__ void k_scatter(Leaves L, const int8_t* __restrict__ eff, const int* __restrict__ off, int ncap,
                          int* __restrict__ nlevel, int* __restrict__ nidx, int* __restrict__ kind,
                          int* __restrict__ src, int* __restrict__ child) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= L.n) return;
  const int e = eff[k], l = L.level[k], o = off[k];
  int ix[D], cnum = 0;
  for (int d = 0; d < D; ++d) { ix[d] = L.idx[d * L.cap + k]; cnum |= (ix[d] & 1) << d; }
  if (e == 0) {
    if (o >= ncap) return;
    nlevel[o] = l;
    for (int d = 0; d < D; ++d) nidx[d * ncap + o] = ix[d];
    kind[o] = 0; src[o] = k; child[o] = 0;
  } else if (e == 1) {
    for (int c = 0; c < (1 << D); ++c) {
      if (o + c >= ncap) return;
      nlevel[o + c] = l + 1;
      for (int d = 0; d < D; ++d) nidx[d * ncap + o + c] = 2 * ix[d] + ((c >> d) & 1);
      kind[o + c] = 1; src[o + c] = k; child[o + c] = c;
    }
  } else if (cnum == 0) {
    if (o >= ncap) return;
    nlevel[o] = l - 1;
    for (int d = 0; d < D; ++d) nidx[d * ncap + o] = ix[d] >> 1;
    kind[o] = 2; src[o] = k; child[o] = 0;
  }
}

// ------------------------------------------------------- remap (Sec. 3.2)
// Gather the new rows (copy or pairwise mean of 2^D brothers) and the
// moments W' of the result.
template <int D, typename T>
__device__ __forceinline__ void d_remap_gather(Geo g, Leaves Lo, Leaves Ln, const int* __restrict__ kind,
                                               const int* __restrict__ src, const T* __restrict__ vin,
                                               T* __restrict__ vout, double* __restrict__ momp, int bx) {
#pragma clang fp contract(off)
  constexpr int P = Cfg<D>::P, N = D + 2;
  __shared__ double red[4 * N];
  const int i = bx;
  const size_t cso = (size_t)g.nc * Lo.ld, csn = (size_t)g.nc * Ln.ld;
  double acc[N];
  for (int m = 0; m < N; ++m) acc[m] = 0.0;
  // four leaves per thread in flight: the source indices and leaf data of
  // the group first, then every leaf's first source value, and only then
  // the other children of merged leaves, the stores and the sums (a leaf at
  // a time made each row read wait on its index load).  The sums keep the
  // order of one leaf after another; a slot past the end re-reads the last
  // leaf and is dropped.
  constexpr int U = 4;
  for (int j0 = threadIdx.x; j0 < Ln.n; j0 += U * BLOCK) {
    int kk[U];
    bool mg[U];
    double xi[U][D], A[U];
    T v[U][P];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int j = min(j0 + t * BLOCK, Ln.n - 1);
      kk[t] = src[j];
      mg[t] = kind[j] == 2;
      int u[D];
      leaf_load<D>(Ln, j, xi[t], A[t], u);
    }
#pragma unroll
    for (int t = 0; t < U; ++t)
#pragma unroll
      for (int p = 0; p < P; ++p) v[t][p] = vin[p * cso + (size_t)i * Lo.ld + kk[t]];
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int j = j0 + t * BLOCK;
      if (j >= Ln.n) break;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if (mg[t]) {
          const T* r = vin + p * cso + (size_t)i * Lo.ld + kk[t];
          if (D == 2) {
            v[t][p] = ((v[t][p] + r[1]) + (r[2] + r[3])) * (T)0.25;
          } else {
            v[t][p] = (((v[t][p] + r[1]) + (r[2] + r[3])) + ((r[4] + r[5]) + (r[6] + r[7]))) * (T)0.125;
          }
        }
        vout[p * csn + (size_t)i * Ln.ld + j] = v[t][p];
      }
      double xi2 = 0.0;
      for (int d = 0; d < D; ++d) xi2 += xi[t][d] * xi[t][d];
      mom_acc<D>(acc, A[t], xi[t], xi2, (double)v[t][0], P == 2 ? (double)v[t][P - 1] : 0.0);
    }
  }
  block_sum<N>(acc, red);
  if (threadIdx.x == 0)
    for (int m = 0; m < N; ++m) momp[(size_t)i * N + m] = acc[m];
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void k_remap_gather(Geo g, Leaves Lo, Leaves Ln, const int* __restrict__ kind,
                             const int* __restrict__ src, const T* __restrict__ vin, T* __restrict__ vout,
                             double* __restrict__ momp) {
  d_remap_gather<D, T>(g, Lo, Ln, kind, src, vin, vout, momp, blockIdx.x);
}

// Conservation correction of Sec. 3.3: f = f' + g_eq(W) - g_eq(W'), then
// (mode 2) the closure that restores M[f] = W.  In place on the new rows.
// With mom non-null, also the moments and heat flux of the corrected rows
// (those of d_cell_moments: same leaf order per thread, same sums).
template <int D, typename T>
__device__ __forceinline__ void d_remap_correct(Geo g, Leaves L, VGrid vg, GasP gas, int mode,
                                                const double* __restrict__ W, const double* __restrict__ momp,
                                                T* __restrict__ vdf, int* __restrict__ bad, double* __restrict__ mom,
                                                double* __restrict__ q, int bx) {
  constexpr int P = Cfg<D>::P, N = D + 2, NS = Cfg<D>::NS;
  extern __shared__ double lds[];
  double* tabA = lds;
  double* tabB = lds + D * vg.numax;
  __shared__ double red[4 * (2 * N + NS)];
  __shared__ double parA[NPAR], parB[NPAR];
  __shared__ double lam[N];
  __shared__ ClosureWork<D> cw;
  const int i = bx;
  if (threadIdx.x == 0) {
    double rho, U[D], T_;
    if (!prim_from_W<D>(W + (size_t)i * N, gas, rho, U, T_)) atomicMin(bad, i);
    eq_record<D>(parA, rho, U, T_, nullptr, gas);
    if (!prim_from_W<D>(momp + (size_t)i * N, gas, rho, U, T_)) atomicMin(bad, i);
    eq_record<D>(parB, rho, U, T_, nullptr, gas);
  }
  __syncthreads();
  build_tab<D>(tabA, parA, vg);
  build_tab<D>(tabB, parB, vg);
  __syncthreads();
  if (mode == 2) {
    double acc[2 * N + NS];
    for (int m = 0; m < 2 * N + NS; ++m) acc[m] = 0.0;
    for (int k = threadIdx.x; k < L.n; k += BLOCK) {
      double xi[D], A;
      int u[D];
      leaf_load<D>(L, k, xi, A, u);
      const double ga = maxw<D>(parA, tabA, vg.numax, u), gb = maxw<D>(parB, tabB, vg.numax, u);
      double c[D], c2 = 0.0, xi2 = 0.0;
      for (int d = 0; d < D; ++d) { c[d] = xi[d] - parA[P_U + d]; c2 += c[d] * c[d]; xi2 += xi[d] * xi[d]; }
      mom_acc<D>(acc, A, xi, xi2, ga, D == 2 ? parA[P_RT] * ga : 0.0);
      mom_acc<D>(acc + N, A, xi, xi2, gb, D == 2 ? parB[P_RT] * gb : 0.0);
      gram_acc<D>(acc + 2 * N, A * ga, c, c2);
    }
    block_sum<2 * N + NS>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int m = 0; m < NS; ++m) cw.S[m] = acc[2 * N + m];
      gram_to_J<D>(cw.S, parA, cw.J);
#pragma unroll
      for (int m = 0; m < N; ++m)
        cw.b[m] = W[(size_t)i * N + m] - (momp[(size_t)i * N + m] + acc[m] - acc[N + m]);
      if (!solve_small<N>(cw.J, cw.b, cw.x)) { atomicMin(bad, i); for (int m = 0; m < N; ++m) cw.x[m] = 0.0; }
      for (int m = 0; m < N; ++m) lam[m] = cw.x[m];
    }
  } else if (threadIdx.x < N) {
    lam[threadIdx.x] = 0.0;
  }
  __syncthreads();
  const size_t cs = (size_t)g.nc * L.ld;
  double U[D];
#pragma unroll
  for (int d = 0; d < D; ++d) U[d] = W[(size_t)i * N + 1 + d] / W[(size_t)i * N];
  double macc[N + D];
#pragma unroll
  for (int m = 0; m < N + D; ++m) macc[m] = 0.0;
  for (int k = threadIdx.x; k < L.n; k += BLOCK) {
    double xi[D], A;
    int u[D];
    leaf_load<D>(L, k, xi, A, u);
    const double ga = maxw<D>(parA, tabA, vg.numax, u), gb = maxw<D>(parB, tabB, vg.numax, u);
    double c2 = 0.0, poly = lam[0];
    for (int d = 0; d < D; ++d) {
      const double c = xi[d] - parA[P_U + d];
      c2 += c * c;
      poly += lam[1 + d] * c;
    }
    poly += lam[D + 1] * c2;
    T* r = vdf + (size_t)i * L.ld + k;
    const T G = (T)(ld_(r) + (ga - gb) + poly * ga);
    r[0] = G;
    T H = 0;
    if (P == 2) {
      H = (T)(ld_(r + cs) + (parA[P_RT] * ga - parB[P_RT] * gb) + poly * parA[P_RT] * ga);
      r[cs] = H;
    }
    if (mom) state_mom_acc<D>(macc, xi, A, U, (double)G, (double)H);
  }
  if (mom) {
    block_sum<N + D>(macc, red);
    if (threadIdx.x == 0) {
      for (int m = 0; m < N; ++m) mom[(size_t)i * N + m] = macc[m];
      for (int d = 0; d < D; ++d) q[(size_t)i * D + d] = macc[N + d];
    }
  }
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void k_remap_correct(Geo g, Leaves L, VGrid vg, GasP gas, int mode,
                             const double* __restrict__ W, const double* __restrict__ momp, T* __restrict__ vdf,
                             int* __restrict__ bad, double* __restrict__ mom, double* __restrict__ q) {
  d_remap_correct<D, T>(g, L, vg, gas, mode, W, momp, vdf, bad, mom, q, blockIdx.x);
}

// -------------------------------------------------- residual, totals, fields
template <int D>
__global__ __launch_bounds__(BLOCK) void k_residual(int nc, const double* __restrict__ W, const double* __restrict__ Wn,
                                                     double invdt, double* __restrict__ out) {
  constexpr int N = D + 2;
  __shared__ double red[4 * N];
  double acc[N];
  for (int m = 0; m < N; ++m) acc[m] = 0.0;
  for (int i = threadIdx.x; i < nc; i += BLOCK)
    for (int m = 0; m < N; ++m) {
      const double d = Wn[(size_t)i * N + m] - W[(size_t)i * N + m];
      acc[m] += d * d;
    }
  block_sum<N>(acc, red);
  if (threadIdx.x == 0)
    for (int m = 0; m < N; ++m) out[m] = sqrt(acc[m]) * invdt;
}

template <int D>
__global__ __launch_bounds__(BLOCK) void k_totals(int nc, const double* __restrict__ vol, const double* __restrict__ W,
                                                   double* __restrict__ out) {
  // vol == nullptr: rows of W summed as they are (a second reduction level)
  constexpr int N = D + 2;
  __shared__ double red[4 * N];
  double acc[N];
  for (int m = 0; m < N; ++m) acc[m] = 0.0;
  for (int i = threadIdx.x; i < nc; i += BLOCK)
    for (int m = 0; m < N; ++m) acc[m] += (vol ? vol[i] : 1.0) * W[(size_t)i * N + m];
  block_sum<N>(acc, red);
  if (threadIdx.x == 0)
    for (int m = 0; m < N; ++m) out[m] = acc[m];
}

// Partial sums of V_i W_i over consecutive blocks of per cells: block b
// writes row b of part (N doubles).
template <int D>
__global__ __launch_bounds__(BLOCK) void k_totals_part(int nc, int per, const double* __restrict__ vol,
                                                        const double* __restrict__ W, double* __restrict__ part) {
  constexpr int N = D + 2;
  __shared__ double red[4 * N];
  double acc[N];
  for (int m = 0; m < N; ++m) acc[m] = 0.0;
  const int i0 = blockIdx.x * per, i1 = min(nc, i0 + per);
  for (int i = i0 + threadIdx.x; i < i1; i += BLOCK)
    for (int m = 0; m < N; ++m) acc[m] += vol[i] * W[(size_t)i * N + m];
  block_sum<N>(acc, red);
  if (threadIdx.x == 0)
    for (int m = 0; m < N; ++m) part[(size_t)blockIdx.x * N + m] = acc[m];
}

template <int D>
__global__ void k_fields(int nc, GasP gas, const double* __restrict__ W, const double* __restrict__ q,
                         double* __restrict__ out) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= nc) return;
  double rho, U[D], T;
  prim_from_W<D>(W + (size_t)i * (D + 2), gas, rho, U, T);
  double* o = out + (size_t)i * (2 * D + 2);
  o[0] = rho;
  for (int d = 0; d < D; ++d) o[1 + d] = U[d];
  o[1 + D] = T;
  for (int d = 0; d < D; ++d) o[2 + D + d] = q[(size_t)i * D + d];
}

}  // namespace avs

namespace avs {

// ----------------------------------------------------------- batched form
// Many independent cases advance in the same launches: one launch per step
// kernel covers the workgroups of every case.  Per-case arguments live in
// device memory (two orientations: even and odd steps swap the state
// buffers), and prefix sums of per-case workgroup counts map a workgroup to
// its case, so the launch sequence can be captured once in a graph.
template <typename T>
struct CaseArgs {
  Geo g;
  Leaves L;
  VGrid vg;
  GasP gas;
  double h, dt;
  const T* vin;
  T* vout;
  T* fv;
  const double* bden;
  const double* bfin;
  double* fpar;
  double* F;
  const double* W;
  double* Wn;
  double* q;
  double* tpar;
  double* lam;
  const double* bcpair;
  double* mom;
  int* bad;
  double* fmom;    // face-moment partials of pass A [nf][2][nchs][NM]
  int nchs;        // their chunk stride
  int chunk, gx;   // pass A: leaves per workgroup, round_up(nc, 8)
};

enum { BK_PASSA, BK_FACEQ, BK_MACRO, BK_TARGET, BK_PASSC, BK_N };

// Largest c with off[c] <= b (off has ncase + 1 increasing entries).
__device__ __forceinline__ int find_case(const int* __restrict__ off, int ncase, int b) {
  int lo = 0, hi = ncase - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Pointers read from device memory are generic to the compiler; the batched
// kernels declare every pointer of a case record global so that uniform
// loads through it become scalar loads, as for kernel arguments.
template <typename E>
__device__ __forceinline__ E* gptr(E* p) {
  typedef __attribute__((address_space(1))) E GE;
  GE* q = (GE*)(uintptr_t)p;
  return (E*)q;
}
#define AVS_G(x) x = gptr(x)
__device__ __forceinline__ Geo global_geo(Geo g) {
  AVS_G(g.order); AVS_G(g.vol); AVS_G(g.eps2); AVS_G(g.dtv); AVS_G(g.nslot); AVS_G(g.s_face); AVS_G(g.s_nbr);
  AVS_G(g.s_sig); AVS_G(g.s_sigA); AVS_G(g.s_d); AVS_G(g.s_dx); AVS_G(g.s_lsq); AVS_G(g.f_L); AVS_G(g.f_R);
  AVS_G(g.f_sL); AVS_G(g.f_sR); AVS_G(g.f_nrm); AVS_G(g.f_int); AVS_G(g.f_bnd); AVS_G(g.bc_kind); AVS_G(g.bc_prim);
  return g;
}
__device__ __forceinline__ Leaves global_leaves(Leaves L) {
  AVS_G(L.level); AVS_G(L.idx); AVS_G(L.u); AVS_G(L.xi); AVS_G(L.w);
  AVS_G(L.xd[0]); AVS_G(L.xd[1]); AVS_G(L.xd[2]); AVS_G(L.ud[0]); AVS_G(L.ud[1]); AVS_G(L.ud[2]);
  return L;
}
#undef AVS_G

template <int D, typename T>
__global__ __launch_bounds__(passA_threads<D>(), (passA_waves<D, T>())) void kb_passA(const CaseArgs<T>* __restrict__ args,
                                                                       const int* __restrict__ off, int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const CaseArgs<T>* a = args + c;
  const int lb = blockIdx.x - off[c];
  d_passA<D, T>(global_geo(a->g), global_leaves(a->L), gptr(a->vin), gptr(a->bcpair), a->h, gptr(a->fv),
                gptr(a->fmom), a->nchs, a->chunk, lb % a->gx, lb / a->gx);
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void kb_face_eq(const CaseArgs<T>* __restrict__ args, const int* __restrict__ off,
                                                   int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const CaseArgs<T>* a = args + c;
  d_face_eq<D, T>(global_geo(a->g), global_leaves(a->L), a->vg, a->gas, a->h, gptr(a->bden), gptr(a->bfin),
                  gptr(a->fmom), a->nchs, (a->L.n + a->chunk - 1) / a->chunk, gptr(a->fpar), gptr(a->F),
                  gptr(a->bad), blockIdx.x - off[c]);
}

template <int D, typename T>
__global__ void kb_macro(const CaseArgs<T>* __restrict__ args, const int* __restrict__ off, int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const CaseArgs<T>* a = args + c;
  d_macro<D>(global_geo(a->g), a->gas, a->dt, gptr(a->F), gptr(a->W), gptr(a->Wn), gptr(a->q), gptr(a->tpar),
             gptr(a->bad), blockIdx.x - off[c], 0);
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void kb_target(const CaseArgs<T>* __restrict__ args, const int* __restrict__ off,
                                                  int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const CaseArgs<T>* a = args + c;
  d_target<D, T>(global_geo(a->g), global_leaves(a->L), a->vg, gptr(a->tpar), gptr(a->Wn), gptr(a->lam), gptr(a->bad),
                 blockIdx.x - off[c], 0);
}

// TWO: two leaves' loads in flight per thread (the batched tuner picks)
template <int D, typename T, bool TWO = passc_two_leaves<D, T>()>
__global__ __launch_bounds__(BLOCK, (waves_hint<D, T>())) void kb_passC(const CaseArgs<T>* __restrict__ args,
                                                                       const int* __restrict__ off, int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const CaseArgs<T>* a = args + c;
  d_passC<D, T, false, TWO>(global_geo(a->g), global_leaves(a->L), a->vg, gptr(a->vin), gptr(a->fv), gptr(a->vout), gptr(a->fpar),
                gptr(a->tpar), gptr(a->lam), gptr(a->mom), gptr(a->q), blockIdx.x - off[c]);
}


// ------------------------------------------- batched remap (all members)
// One record per member for the remap of a batched adaptation: the old and
// new leaves, the state buffers (in: the old rows, out: the new), and what
// the boundary tables and moments of the new leaves need.
template <typename T>
struct RemapArgs {
  Geo g;
  Leaves Lo, Ln;
  VGrid vg;
  GasP gas;
  const int* pkind;
  const int* psrc;
  const T* vin;
  T* vout;
  double* momp;
  const double* W;
  double* mom;
  double* q;
  int* bad;
  double* bcpair;
  double* bden;
  double* bfin;
  int nbl;         // ceil(new leaves / BLOCK): blocks per boundary condition of the pair tables
};

enum { BR_GATHER, BR_CORRECT, BR_PAIRS, BR_BND, BR_MOM, BR_N };

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void kb_remap_gather(const RemapArgs<T>* __restrict__ args,
                                                         const int* __restrict__ off, int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const RemapArgs<T>* a = args + c;
  d_remap_gather<D, T>(global_geo(a->g), global_leaves(a->Lo), global_leaves(a->Ln), gptr(a->pkind), gptr(a->psrc),
                       gptr(a->vin), gptr(a->vout), gptr(a->momp), blockIdx.x - off[c]);
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void kb_remap_correct(const RemapArgs<T>* __restrict__ args,
                                                          const int* __restrict__ off, int ncase, int mode) {
  const int c = find_case(off, ncase, blockIdx.x);
  const RemapArgs<T>* a = args + c;
  d_remap_correct<D, T>(global_geo(a->g), global_leaves(a->Ln), a->vg, a->gas, mode, gptr(a->W), gptr(a->momp),
                        gptr(a->vout), gptr(a->bad), gptr(a->mom), gptr(a->q), blockIdx.x - off[c]);
}

template <int D, typename T>
__global__ void kb_bc_pairs(const RemapArgs<T>* __restrict__ args, const int* __restrict__ off, int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const RemapArgs<T>* a = args + c;
  const int lb = blockIdx.x - off[c];
  const Geo g = global_geo(a->g);
  d_bc_pairs<D>(global_leaves(a->Ln), a->gas, g.nbc, g.bc_kind, g.bc_prim, gptr(a->bcpair), lb % a->nbl, lb / a->nbl);
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void kb_bnd_tables(const RemapArgs<T>* __restrict__ args,
                                                       const int* __restrict__ off, int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const RemapArgs<T>* a = args + c;
  d_bnd_tables<D>(global_geo(a->g), global_leaves(a->Ln), gptr(a->bcpair), gptr(a->bden), gptr(a->bfin),
                  blockIdx.x - off[c]);
}

template <int D, typename T>
__global__ __launch_bounds__(BLOCK) void kb_cell_moments(const RemapArgs<T>* __restrict__ args,
                                                         const int* __restrict__ off, int ncase) {
  const int c = find_case(off, ncase, blockIdx.x);
  const RemapArgs<T>* a = args + c;
  d_cell_moments<D, T>(global_geo(a->g), global_leaves(a->Ln), gptr(a->vout), gptr(a->W), gptr(a->mom), gptr(a->q),
                       blockIdx.x - off[c]);
}

}  // namespace avs
