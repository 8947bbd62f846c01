// Internal definitions shared by the host side of libavs and its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace avs {

constexpr int BLOCK = 256;       // threads per workgroup (4 wave64)
constexpr int MAXF2 = 4;         // max faces per cell, 2-D
constexpr int MAXF3 = 6;         // max faces per cell, 3-D
constexpr int NM2 = 9;           // raw face moments, 2-D: m0, m1[2], m2[3], e, e1[2]
constexpr int NM3 = 14;          // raw face moments, 3-D: m0, m1[3], m2[6], e, e1[3]
constexpr int NPAR = 16;         // doubles per equilibrium parameter record
constexpr int CRIT_CELLS = 256;  // cells per criterion partial
#ifndef AVS_CHUNK
#define AVS_CHUNK 8192
#endif
constexpr int CHUNK = AVS_CHUNK;  // leaves per workgroup of pass A
constexpr int CHUNK_MIN = 512;    // smallest pass-A chunk (sizes the face-moment partials)

// Equilibrium parameter record (face or cell), NPAR doubles:
//   [0] coef = rho (2 pi R T)^(-D/2)   [1..3] U   [4] RT   [5] 1/(2RT)   [6] 1/RT
//   [7..9] q   [10] shk = (1-Pr)/(5 p RT) (0 for BGK)
//   face: [11] a = tau/(tau+h)  [12] b = h/(tau+h)
//   cell: [11] dt/tau           [12] rho  [13] T
//   boundary face: [0] rho_w (wall)
enum { P_COEF = 0, P_U = 1, P_RT = 4, P_I2RT = 5, P_IRT = 6, P_Q = 7, P_SHK = 10, P_A = 11, P_B = 12, P_RHO = 12, P_T = 13 };

struct Geo {
  int D, P, nc, nf, maxf, nbc;
  int n_int, n_bnd;
  const int* order;      // [nc] cells along a space-filling curve of their centres
  const double* vol;     // [nc]
  const double* eps2;    // [nc]  (K V^(1/D))^3
  const double* dtv;     // [nc]  dt / V
  const int* nslot;      // [nc]
  const int* s_face;     // [nc*maxf]
  const int* s_nbr;      // [nc*maxf]   neighbour cell or -1
  const double* s_sig;   // [nc*maxf]   +1 if the cell is the face's L side
  const double* s_sigA;  // [nc*maxf]   sigma * area
  const double* s_d;     // [nc*maxf*D] face midpoint - cell centre (cell frame)
  const double* s_dx;    // [nc*maxf*D] neighbour centre - cell centre (cell frame)
  const double* s_lsq;   // [nc*maxf*D] least-squares coefficients
  const int* f_L;        // [nf]
  const int* f_R;        // [nf]  >=0 cell, else -1-bc
  const int* f_sL;       // [nf]  slot of the face in L
  const int* f_sR;       // [nf]  slot in R (interior)
  const double* f_nrm;   // [nf*D]
  const int* f_int;      // [n_int] interior faces
  const int* f_bnd;      // [n_bnd] boundary faces
  const int* bc_kind;    // [nbc]
  const double* bc_prim; // [nbc*(D+2)]
};

struct Leaves {
  int n;       // leaves
  int ld;      // VDF row stride
  int cap;     // SoA stride of the arrays below
  const int* level;   // [cap]
  const int* idx;     // [D*cap]
  const int* u;       // [D*cap] centre on the half-finest grid: (2 idx + 1) << (Lmax - level)
  const double* xi;   // [D*cap]
  const double* w;    // [cap]
  // rows of each dimension, xi + d cap and u + d cap (the first row beyond
  // D): passed as such, a load is a scalar base plus the lane's 32-bit
  // offset, where base + d cap + offset became a 64-bit vector add per load
  const double* xd[3];
  const int* ud[3];
};

struct VGrid {          // the half-finest grid that carries every leaf centre
  int nu[3];
  int numax;
  double x0[3];         // lo
  double hh[3];         // (hi - lo) / (base 2^(Lmax+1))
};

struct GasP {
  double R, Pr, omega, mu_ref, T_ref;
  int model;
  int law;         // viscosity: 0 power law, 1 Sutherland
  double C_s;      // Sutherland constant
};

}  // namespace avs
