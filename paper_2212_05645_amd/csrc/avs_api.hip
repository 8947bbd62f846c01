// Host side of libavs: argument checking, mesh preprocessing, workspace
// layout, kernel sequencing and the extern "C" entry points of avs.h.
#include <algorithm>
#include <cinttypes>
#include <cstdarg>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/avs.h"
#include "avs_kernels.hip"
#include "avs_implicit.hip"
#include "avs_dia.hip"
#include "avs_mlp.hip"

using namespace avs;

namespace {

thread_local std::string g_err;

avs_status fail(avs_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
avs_status fail(avs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Bump allocator over the caller's workspace (base == nullptr: measure only).
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

struct LeafBuf {
  int* level;
  int* idx;
  int* u;
  double* xi;
  double* w;
};

}  // namespace

struct avs_ctx {
  int D, P, maxf, prec;
  int nc, nf, nbc, n_int, n_bnd;
  int64_t cap;
  int lmax, base[3];
  double lo[3], hi[3];
  GasP gas;
  double dt, h, Kv;
  VGrid vg;
  hipStream_t stream;
  int device = 0;         // current device at init: the device of the caller's memory and stream
  bool failed = false;
  std::vector<double> vol_host;

  void* vdf[2];
  void* fv;               // interface buffer: upwind reconstruction per (face, leaf)
  size_t vdf_buf_bytes;
  int cur = 0;

  Geo geo;
  LeafBuf lt[2];
  int lcur = 0;
  int nleaf[2] = {0, 0};
  int ld[2] = {0, 0};

  double *W, *Wn, *q, *mom, *tpar, *lam, *fpar, *F, *bden, *bfin, *bcpair, *momp, *res, *tot;
  double* fmom;           // face-moment partials of pass A: [nf+1][2 sides][nchs chunks][NM]
  int nchs;               // chunk stride of fmom: ceil(capacity / CHUNK_MIN)
  double *cc, *crit_part, *Mk, *probe_cc, *probe_prim;
  int8_t *raw, *eff;
  int *cnt, *off, *pkind, *psrc, *pchild, *bad;
  double *rA, *irhs, *idiag, *dW;                // implicit predictor: r per face, rhs, diagonal, increment
  int64_t leaf_gen = 0;                          // bumped whenever the leaf set changes
  int* col_cells;                                // cells in colour-major order
  std::vector<int> col_off;                      // colour c holds col_cells[col_off[c] .. col_off[c+1])
  uint16_t* feat = nullptr;                      // learned proposal (2-D): feature rows [cap][32]
  double *quant = nullptr, *tprobe = nullptr, *terr = nullptr;
  int ngrp;
  int nprobe_max = 64;
  int plan_n = 0;
  bool plan_valid = false;
  // the diatomic state whose adaptation made the current plan (nullptr: a
  // monatomic adaptation made it); a diatomic remap needs its own plan,
  // whose leaf count its rows were checked against
  const void* plan_owner = nullptr;
  // separated zone (Sec. 3.5): a floor on the flags of every adaptation;
  // sep_level < 0 when unset
  double sep_lo = 0.0, sep_hi = 0.0;
  int sep_level = -1;

  // optional per-kernel timing with HIP events (measurement only)
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<std::pair<int, size_t>> evrec;   // (kernel id, index of its start event)

  Leaves leaves(int t) const {
    Leaves L;
    L.n = nleaf[t];
    L.ld = ld[t];
    L.cap = (int)cap;
    L.level = lt[t].level;
    L.idx = lt[t].idx;
    L.u = lt[t].u;
    L.xi = lt[t].xi;
    L.w = lt[t].w;
    for (int d = 0; d < 3; ++d) {
      L.xd[d] = lt[t].xi + (d < D ? (size_t)d * cap : 0);
      L.ud[d] = lt[t].u + (d < D ? (size_t)d * cap : 0);
    }
    return L;
  }
  size_t esize() const { return prec == AVS_FP32 ? 4 : 8; }
};

namespace {

enum KernelId { K_PASSA, K_FACE, K_FACE_EQFLUX, K_MACRO, K_TARGET, K_PASSC, K_RESIDUAL, K_CRITERION,
                K_FLAGS, K_REMAP_GATHER, K_REMAP_CORRECT, K_BC_TABLES, K_MOMENTS, K_INIT, K_LEARNED,
                K_IMP_MACRO, K_IMP_RES, K_IMP_MICRO, K_NKERNELS };
const char* const kKernelNames[K_NKERNELS] = {"passA", "face", "face_eqflux", "macro", "target", "passC",
                                              "residual", "criterion", "flags_plan", "remap_gather",
                                              "remap_correct", "bc_tables", "moments", "init_vdf", "learned",
                                              "imp_macro", "imp_res", "imp_micro"};

hipEvent_t next_event(avs_ctx* ctx) {
  if (ctx->evused == ctx->evpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->evpool.push_back(e);
  }
  return ctx->evpool[ctx->evused++];
}

// Brackets a group of launches with two events when profiling is on.
struct ProfScope {
  avs_ctx* ctx;
  int id;
  ProfScope(avs_ctx* c, int k) : ctx(c), id(k) {
    if (ctx->prof) {
      const size_t at = ctx->evused;
      hipEvent_t a = next_event(ctx);
      hipEvent_t b = next_event(ctx);
      if (a && b && hipEventRecord(a, ctx->stream) == hipSuccess) ctx->evrec.push_back({id, at});
      (void)b;
    }
  }
  ~ProfScope() {
    if (ctx->prof && !ctx->evrec.empty() && ctx->evrec.back().first == id)
      (void)hipEventRecord(ctx->evpool[ctx->evrec.back().second + 1], ctx->stream);
  }
};

#define CK(expr)                                                                                   \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      if (ctx) ctx->failed = true;                                                                 \
      return fail(AVS_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    }                                                                                              \
  } while (0)

#define CKL()                                                                                      \
  do {                                                                                             \
    hipError_t e_ = hipGetLastError();                                                             \
    if (e_ != hipSuccess) {                                                                        \
      if (ctx) ctx->failed = true;                                                                 \
      return fail(AVS_E_HIP, "kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
    }                                                                                              \
  } while (0)

avs_status check_args(const avs_vspace* vs, const avs_pmesh* pm, const avs_opts* op) {
  if (!vs || !pm || !op) return fail(AVS_E_INVALID, "null descriptor");
  if (vs->dim != 2 && vs->dim != 3) return fail(AVS_E_INVALID, "vspace.dim must be 2 or 3 (got %d)", vs->dim);
  if (pm->dim != vs->dim) return fail(AVS_E_INVALID, "pmesh.dim %d != vspace.dim %d", pm->dim, vs->dim);
  if (vs->max_level < 0 || vs->max_level > 12) return fail(AVS_E_INVALID, "max_level %d outside [0, 12]", vs->max_level);
  int64_t nroots = 1;
  for (int d = 0; d < vs->dim; ++d) {
    if (vs->base[d] < 1 || vs->base[d] > 4096) return fail(AVS_E_INVALID, "base[%d] = %d outside [1, 4096]", d, vs->base[d]);
    if (!(vs->hi[d] > vs->lo[d])) return fail(AVS_E_INVALID, "velocity box empty on axis %d", d);
    nroots *= vs->base[d];
    if (((int64_t)vs->base[d] << (vs->max_level + 1)) > (1 << 20))
      return fail(AVS_E_INVALID, "base[%d] * 2^max_level too large", d);
  }
  if (vs->leaf_capacity < nroots) return fail(AVS_E_INVALID, "leaf_capacity %" PRId64 " < number of roots %" PRId64, vs->leaf_capacity, nroots);
  if (vs->leaf_capacity > (1 << 26)) return fail(AVS_E_INVALID, "leaf_capacity too large");
  if (pm->ncells < 1 || pm->ncells > (1 << 28)) return fail(AVS_E_INVALID, "ncells %" PRId64 " out of range", pm->ncells);
  if (pm->nfaces < 0 || pm->nfaces > (1 << 29)) return fail(AVS_E_INVALID, "nfaces %" PRId64 " out of range", pm->nfaces);
  if (op->precision != AVS_FP64 && op->precision != AVS_FP32) return fail(AVS_E_INVALID, "precision must be AVS_FP64 or AVS_FP32");
  if (!(op->dt > 0.0)) return fail(AVS_E_INVALID, "dt must be > 0");
  if (!(op->venkat_K >= 0.0)) return fail(AVS_E_INVALID, "venkat_K must be >= 0");
  return AVS_OK;
}

int numax_of(const avs_vspace* vs) {
  int m = 0;
  for (int d = 0; d < vs->dim; ++d) m = std::max(m, vs->base[d] << (vs->max_level + 1));
  return m;
}

// Carve every device array of a context; with c.base == nullptr only sizes.
void carve(avs_ctx& x, Carver& c) {
  const int D = x.D, N = D + 2;
  const size_t nc = x.nc, nf = x.nf, cap = x.cap, mf = x.maxf;
  x.geo.order = c.take<int>(nc);
  x.geo.vol = c.take<double>(nc);
  x.geo.eps2 = c.take<double>(nc);
  x.geo.dtv = c.take<double>(nc);
  x.geo.nslot = c.take<int>(nc);
  x.geo.s_face = c.take<int>(nc * mf);
  x.geo.s_nbr = c.take<int>(nc * mf);
  x.geo.s_sig = c.take<double>(nc * mf);
  x.geo.s_sigA = c.take<double>(nc * mf);
  x.geo.s_d = c.take<double>(nc * mf * D);
  x.geo.s_dx = c.take<double>(nc * mf * D);
  x.geo.s_lsq = c.take<double>(nc * mf * D);
  x.geo.f_L = c.take<int>(nf + 1);
  x.geo.f_R = c.take<int>(nf + 1);
  x.geo.f_sL = c.take<int>(nf + 1);
  x.geo.f_sR = c.take<int>(nf + 1);
  x.geo.f_nrm = c.take<double>((nf + 1) * D);
  x.geo.f_int = c.take<int>(nf + 1);
  x.geo.f_bnd = c.take<int>(nf + 1);
  x.geo.bc_kind = c.take<int>(x.nbc + 1);
  x.geo.bc_prim = c.take<double>((x.nbc + 1) * N);
  for (int t = 0; t < 2; ++t) {
    x.lt[t].level = c.take<int>(cap);
    x.lt[t].idx = c.take<int>(cap * D);
    x.lt[t].u = c.take<int>(cap * D);
    x.lt[t].xi = c.take<double>(cap * D);
    x.lt[t].w = c.take<double>(cap);
  }
  x.W = c.take<double>(nc * N);
  x.Wn = c.take<double>(nc * N);
  x.q = c.take<double>(nc * D);
  x.mom = c.take<double>(nc * N);
  x.tpar = c.take<double>(nc * NPAR);
  x.lam = c.take<double>(nc * N);
  x.fpar = c.take<double>((nf + 1) * NPAR);
  x.nchs = (int)((cap + CHUNK_MIN - 1) / CHUNK_MIN);
  x.fmom = c.take<double>((nf + 1) * 2 * (size_t)x.nchs * (D == 2 ? NM2 : NM3));
  x.F = c.take<double>((nf + 1) * N);
  x.bden = c.take<double>(nf + 1);
  x.bfin = c.take<double>((nf + 1) * N);
  x.bcpair = c.take<double>((size_t)(x.nbc + 1) * x.P * cap);
  x.momp = c.take<double>(nc * N);
  x.res = c.take<double>(N);
  x.tot = c.take<double>(N);
  x.cc = c.take<double>(nc * N);
  x.ngrp = (int)((nc + CRIT_CELLS - 1) / CRIT_CELLS);
  x.crit_part = c.take<double>((size_t)x.ngrp * cap);
  x.Mk = c.take<double>(cap);
  x.probe_cc = c.take<double>((size_t)x.nprobe_max * N);
  x.probe_prim = c.take<double>((size_t)x.nprobe_max * N);
  x.raw = c.take<int8_t>(cap);
  x.eff = c.take<int8_t>(cap);
  x.cnt = c.take<int>(cap);
  x.off = c.take<int>(cap + 1);
  x.pkind = c.take<int>(cap);
  x.psrc = c.take<int>(cap);
  x.pchild = c.take<int>(cap);
  x.bad = c.take<int>(4);
  x.rA = c.take<double>(nf + 1);
  x.irhs = c.take<double>(nc * N);
  x.idiag = c.take<double>(nc);
  x.dW = c.take<double>(nc * N);
  x.col_cells = c.take<int>(nc);
  if (D == 2) {
    x.feat = c.take<uint16_t>(cap * mlp::NINP);
    x.quant = c.take<double>(24);
    x.tprobe = c.take<double>((size_t)(x.nprobe_max + 8) * 4);
    x.terr = c.take<double>((size_t)x.nprobe_max + 8);
  }
}

void fill_dims(avs_ctx& x, const avs_vspace* vs, const avs_pmesh* pm, const avs_opts* op) {
  x.D = vs->dim;
  x.P = x.D == 2 ? 2 : 1;
  x.maxf = x.D == 2 ? MAXF2 : MAXF3;
  x.prec = op->precision;
  x.nc = (int)pm->ncells;
  x.nf = (int)pm->nfaces;
  x.nbc = pm->nbc;
  x.cap = round_up(vs->leaf_capacity, 64);
}

// Morton key of a leaf's lower corner on the finest grid (x lowest bit).
uint64_t morton(int D, int lmax, int level, const int* ix) {
  uint64_t key = 0;
  const int bits = 64 / D;
  for (int b = 0; b < bits; ++b)
    for (int d = 0; d < D; ++d) {
      const uint64_t X = (uint64_t)ix[d] << (lmax - level);
      key |= ((X >> b) & 1ull) << (D * b + d);
    }
  return key;
}

// Pseudo-inverse of a symmetric positive semi-definite DxD matrix (Jacobi).
void pinv_sym(int D, const double* M, double* out) {
  double a[3][3], v[3][3];
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) { a[i][j] = M[i * D + j]; v[i][j] = i == j; }
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < D; ++i)
      for (int j = i + 1; j < D; ++j) off += a[i][j] * a[i][j];
    if (off < 1e-300) break;
    for (int p = 0; p < D; ++p)
      for (int q = p + 1; q < D; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < D; ++k) {
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < D; ++k) {
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < D; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - s * vkq;
          v[k][q] = s * vkp + c * vkq;
        }
      }
  }
  double emax = 0.0;
  for (int i = 0; i < D; ++i) emax = std::max(emax, fabs(a[i][i]));
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int k = 0; k < D; ++k)
        if (a[k][k] > 1e-12 * emax) s += v[i][k] * v[j][k] / a[k][k];
      out[i * D + j] = s;
    }
}

// W = (rho, rho U, rho|U|^2/2 + 3/2 rho R T); same operation order as the oracle.
void conserved_host(int D, double R, const double* prim, double* W) {
#pragma clang fp contract(off)
  const double rho = prim[0];
  double ss = prim[1] * prim[1];
  for (int d = 1; d < D; ++d) ss = ss + prim[1 + d] * prim[1 + d];
  const double ke = 0.5 * rho * ss;
  W[0] = rho;
  for (int d = 0; d < D; ++d) W[1 + d] = rho * prim[1 + d];
  W[1 + D] = ke + 1.5 * rho * R * prim[1 + D];
}

// Diatomic conserved state (rho, rho U, rho E, rho E_rot) of an equilibrium
// probe (T_t = T_r = T), in the oracle's operation order: rho E_rot = rho R T,
// rho E = rho|U|^2/2 + 3/2 rho R T + rho E_rot.
void conserved_dia_host(int D, double R, const double* prim, double* W) {
#pragma clang fp contract(off)
  const double rho = prim[0], T = prim[1 + D];
  double ss = prim[1] * prim[1];
  for (int d = 1; d < D; ++d) ss = ss + prim[1 + d] * prim[1 + d];
  W[0] = rho;
  for (int d = 0; d < D; ++d) W[1 + d] = rho * prim[1 + d];
  W[2 + D] = rho * R * T;
  W[1 + D] = 0.5 * rho * ss + 1.5 * rho * R * T + W[2 + D];
}

void crit_consts_host(int D, const double* W, double* o) {
#pragma clang fp contract(off)
  const double rho = W[0];
  double U[3];
  for (int d = 0; d < D; ++d) U[d] = W[1 + d] / rho;
  double ke = U[0] * U[0];
  for (int d = 1; d < D; ++d) ke = ke + U[d] * U[d];
  o[0] = rho;
  for (int d = 0; d < D; ++d) o[1 + d] = U[d];
  o[1 + D] = W[1 + D] - 0.5 * rho * ke;
}

template <typename T>
void copy_from_host(std::vector<T>& tmp, const double* src, size_t n) {
  tmp.resize(n);
  for (size_t i = 0; i < n; ++i) tmp[i] = (T)src[i];
}

// ------------------------------------------------------------- launchers
template <int D, typename T>
avs_status launch_init_vdf(avs_ctx* ctx, bool close = true) {
  constexpr int N = D + 2, NS = Cfg<D>::NS;
  const size_t shm = (size_t)(D * ctx->vg.numax + 4 * (N + NS)) * sizeof(double);
  k_init_vdf<D, T><<<ctx->nc, BLOCK, shm, ctx->stream>>>(ctx->geo, ctx->leaves(ctx->lcur), ctx->vg, ctx->gas, ctx->W,
                                                       (T*)ctx->vdf[ctx->cur], ctx->bad, close ? 1 : 0);
  CKL();
  return AVS_OK;
}

template <int D, typename T>
avs_status launch_moments(avs_ctx* ctx) {
  ProfScope ps(ctx, K_MOMENTS);
  k_cell_moments<D, T><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->leaves(ctx->lcur), (const T*)ctx->vdf[ctx->cur],
                                                          ctx->W, ctx->mom, ctx->q);
  CKL();
  return AVS_OK;
}

template <int D>
avs_status launch_bc_tables(avs_ctx* ctx) {
  const Leaves L = ctx->leaves(ctx->lcur);
  ProfScope ps(ctx, K_BC_TABLES);
  if (ctx->nbc > 0) {
    dim3 grid((L.n + BLOCK - 1) / BLOCK, ctx->nbc);
    k_bc_pairs<D><<<grid, BLOCK, 0, ctx->stream>>>(L, ctx->gas, ctx->nbc, ctx->geo.bc_kind, ctx->geo.bc_prim, ctx->bcpair);
    CKL();
  }
  if (ctx->n_bnd > 0) {
    k_bnd_tables<D><<<ctx->n_bnd, BLOCK, 0, ctx->stream>>>(ctx->geo, L, ctx->bcpair, ctx->bden, ctx->bfin);
    CKL();
  }
  return AVS_OK;
}

// Interface stage of a step: reconstruction into the interface buffer,
// interface moments and records, fluxes F_f.
template <int D, typename T>
avs_status launch_interfaces(avs_ctx* ctx) {
  const Leaves L = ctx->leaves(ctx->lcur);
  const int nu = ctx->vg.numax;
  const T* vin = (const T*)ctx->vdf[ctx->cur];
  // pass-A leaves per workgroup: longer chunks in the FP32 form, where a
  // leaf costs about half as much, so that the per-workgroup set-up and
  // reductions keep their share (2-D: 16384 measured 1 % faster than 8192;
  // 3-D: 32768, whole rows of the 20 000-leaf sphere, 4.5 % faster than
  // 16384; FP64 no faster)
  const int chunk = sizeof(T) == 4 ? (D == 3 ? 4 : 2) * CHUNK : CHUNK;
  const int nch = (L.n + chunk - 1) / chunk;
  {
    // reconstruction, interface rows and the faces' moment partials
    ProfScope ps(ctx, K_PASSA);
    const int gx = (int)round_up(ctx->nc, 8);
    k_passA<D, T><<<dim3(gx, nch), passA_threads<D>(), 0, ctx->stream>>>(ctx->geo, L, vin, ctx->bcpair, ctx->h, (T*)ctx->fv,
                                                            ctx->fmom, ctx->nchs, chunk);
    CKL();
  }
  {
    ProfScope ps(ctx, K_FACE_EQFLUX);
    k_face_eq<D, T><<<(ctx->nf + face_batch<D>() - 1) / face_batch<D>(), BLOCK, (size_t)face_batch<D>() * D * nu * sizeof(T),
                      ctx->stream>>>(
        ctx->geo, L, ctx->vg, ctx->gas, ctx->h, ctx->bden, ctx->bfin, ctx->fmom, ctx->nchs, nch, ctx->fpar, ctx->F,
        ctx->bad);
    CKL();
  }
  return AVS_OK;
}

template <int D, typename T>
avs_status launch_step(avs_ctx* ctx, bool last_residual) {
  constexpr int MAXF = Cfg<D>::MAXF;
  const Leaves L = ctx->leaves(ctx->lcur);
  const int nu = ctx->vg.numax;
  const T* vin = (const T*)ctx->vdf[ctx->cur];
  T* vout = (T*)ctx->vdf[ctx->cur ^ 1];
  if (avs_status st = launch_interfaces<D, T>(ctx)) return st;
  {
    ProfScope ps(ctx, K_MACRO);
    k_macro<D><<<(ctx->nc + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->gas, ctx->dt, ctx->F, ctx->W,
                                                                       ctx->Wn, ctx->q, ctx->tpar, ctx->bad);
    CKL();
  }
  {
    ProfScope ps(ctx, K_TARGET);
    k_target<D, T><<<ctx->nc, BLOCK, (size_t)D * nu * sizeof(T), ctx->stream>>>(ctx->geo, L, ctx->vg, ctx->tpar, ctx->Wn,
                                                                               ctx->lam, ctx->bad);
    CKL();
  }
  {
    ProfScope ps(ctx, K_PASSC);
    k_passC<D, T><<<(unsigned)round_up(ctx->nc, 8), BLOCK, (size_t)(MAXF + 1) * D * nu * sizeof(T), ctx->stream>>>(
        ctx->geo, L, ctx->vg, vin, (const T*)ctx->fv, vout, ctx->fpar, ctx->tpar, ctx->lam, ctx->mom, ctx->q);
    CKL();
  }
  if (last_residual) {
    ProfScope ps(ctx, K_RESIDUAL);
    k_residual<D><<<1, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->W, ctx->Wn, 1.0 / ctx->dt, ctx->res);
    CKL();
  }
  std::swap(ctx->W, ctx->Wn);
  ctx->cur ^= 1;
  return AVS_OK;
}

// One implicit step (IUGKS): interfaces as in the explicit step, then the
// PRSGS predictor (n_macro symmetric sweeps, colours up then down), W^{n+1}
// in flux form with the implicit flux of the predicted increment, the
// target from W^{n+1}, the micro right-hand side from pass C,
// n_micro symmetric sweeps of the upwind micro system into the second VDF
// buffer, phi^{n+1} = phi^n + dphi, and the moments of phi^{n+1}.
template <int D, typename T>
avs_status launch_step_implicit(avs_ctx* ctx, int n_macro, int n_micro, T* res, bool last_residual) {
  constexpr int MAXF = Cfg<D>::MAXF;
  const Leaves L = ctx->leaves(ctx->lcur);
  const int nu = ctx->vg.numax;
  const T* vin = (const T*)ctx->vdf[ctx->cur];
  T* dphi = (T*)ctx->vdf[ctx->cur ^ 1];
  const int ncol = (int)ctx->col_off.size() - 1;
  const unsigned gc = (unsigned)((ctx->nc + BLOCK - 1) / BLOCK);
  if (avs_status st = launch_interfaces<D, T>(ctx)) return st;
  {
    ProfScope ps(ctx, K_IMP_MACRO);
    k_imp_rface<D><<<(unsigned)((ctx->nf + BLOCK - 1) / BLOCK), BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->gas, ctx->h, ctx->W,
                                                                                       ctx->fpar, ctx->rA);
    CKL();
    k_imp_rhs<D><<<gc, BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->F, ctx->rA, ctx->irhs, ctx->idiag, ctx->dW);
    CKL();
    for (int sw = 0; sw < n_macro; ++sw)
      for (int t = 0; t < 2 * ncol; ++t) {
        const int c = t < ncol ? t : 2 * ncol - 1 - t;
        const int cnt = ctx->col_off[c + 1] - ctx->col_off[c];
        k_imp_macro<D><<<(unsigned)((cnt + BLOCK - 1) / BLOCK), BLOCK, 0, ctx->stream>>>(
            ctx->geo, ctx->gas, ctx->col_cells + ctx->col_off[c], cnt, ctx->W, ctx->rA, ctx->irhs, ctx->idiag, ctx->dW);
        CKL();
      }
    k_imp_fhat<D><<<(unsigned)((ctx->nf + BLOCK - 1) / BLOCK), BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->gas, ctx->W,
                                                                                      ctx->dW, ctx->rA, ctx->F);
    CKL();
    k_macro<D><<<gc, BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->gas, ctx->dt, ctx->F, ctx->W, ctx->Wn, ctx->q, ctx->tpar,
                                              ctx->bad);
    CKL();
  }
  {
    ProfScope ps(ctx, K_TARGET);
    k_target<D, T><<<ctx->nc, BLOCK, (size_t)D * nu * sizeof(T), ctx->stream>>>(ctx->geo, L, ctx->vg, ctx->tpar, ctx->Wn,
                                                                               ctx->lam, ctx->bad);
    CKL();
  }
  {
    ProfScope ps(ctx, K_IMP_RES);
    k_passC_res<D, T><<<(unsigned)round_up(ctx->nc, 8), BLOCK, (size_t)(MAXF + 1) * D * nu * sizeof(T), ctx->stream>>>(
        ctx->geo, L, ctx->vg, vin, (const T*)ctx->fv, res, ctx->fpar, ctx->tpar, ctx->lam);
    CKL();
  }
  {
    ProfScope ps(ctx, K_IMP_MICRO);
    k_imp_zero<T><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->P, ctx->nc, L, dphi);
    CKL();
    for (int sw = 0; sw < n_micro; ++sw)
      for (int t = 0; t < 2 * ncol; ++t) {
        const int c = t < ncol ? t : 2 * ncol - 1 - t;
        const int cnt = ctx->col_off[c + 1] - ctx->col_off[c];
        k_imp_micro<D, T><<<(unsigned)cnt, BLOCK, 0, ctx->stream>>>(ctx->geo, L, ctx->col_cells + ctx->col_off[c], res,
                                                                     dphi, ctx->tpar, NPAR, P_A);
        CKL();
      }
    k_imp_finish<T><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->P, ctx->nc, L, vin, dphi);
    CKL();
  }
  if (last_residual) {
    ProfScope ps(ctx, K_RESIDUAL);
    k_residual<D><<<1, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->W, ctx->Wn, 1.0 / ctx->dt, ctx->res);
    CKL();
  }
  std::swap(ctx->W, ctx->Wn);
  ctx->cur ^= 1;
  {
    ProfScope ps(ctx, K_MOMENTS);
    k_cell_moments<D, T><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->geo, L, (const T*)ctx->vdf[ctx->cur], ctx->W, ctx->mom,
                                                            ctx->q);
    CKL();
  }
  return AVS_OK;
}

template <int D>
avs_status launch_leaf_geom(avs_ctx* ctx, int t) {
  const int n = ctx->nleaf[t];
  if (n == 0) return AVS_OK;
  k_leaf_geom<D><<<(n + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(
      n, (int)ctx->cap, ctx->lt[t].level, ctx->lt[t].idx, ctx->lt[t].u, ctx->lt[t].xi, ctx->lt[t].w, ctx->vg, ctx->lmax,
      ctx->base[0], ctx->base[1], ctx->base[2], ctx->lo[0], ctx->lo[1], ctx->lo[2], ctx->hi[0], ctx->hi[1], ctx->hi[2]);
  CKL();
  return AVS_OK;
}

// The separated-zone floor on the raw flags, when the context has a zone.
template <int D>
avs_status launch_sep_floor(avs_ctx* ctx, const Leaves& L) {
  if (ctx->sep_level < 0 || L.n == 0) return AVS_OK;
  k_sep_floor<D><<<(L.n + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(
      L, ctx->lmax, ctx->base[0], ctx->base[1], ctx->base[2], ctx->lo[0], ctx->lo[1], ctx->lo[2], ctx->hi[0],
      ctx->hi[1], ctx->hi[2], ctx->sep_lo * ctx->sep_lo, ctx->sep_hi * ctx->sep_hi, ctx->sep_level, ctx->raw);
  CKL();
  return AVS_OK;
}

// Criterion, raw and effective flags, and their scan.  cells == false: the
// criterion runs over the probe states only (step-0 velocity space).
template <int D, typename T>
avs_status launch_adapt(avs_ctx* ctx, double C1, double C2, int nprobe, bool cells = true) {
  const Leaves L = ctx->leaves(ctx->lcur);
  const int nb = (L.n + BLOCK - 1) / BLOCK;
  ProfScope ps(ctx, K_CRITERION);
  if (cells) {
    k_crit_cells<D><<<(ctx->nc + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->W, ctx->cc);
    CKL();
    k_crit_partial<D, T><<<dim3(nb, ctx->ngrp), BLOCK, 0, ctx->stream>>>(L, ctx->nc, (const T*)ctx->vdf[ctx->cur],
                                                                        ctx->cc, ctx->crit_part);
    CKL();
  }
  k_crit_reduce<D><<<nb, BLOCK, 0, ctx->stream>>>(L, cells ? ctx->ngrp : 0, ctx->crit_part, nprobe, ctx->probe_cc,
                                                 ctx->probe_prim, ctx->gas, C1, C2, ctx->lmax, ctx->Mk, ctx->raw);
  CKL();
  if (avs_status st = launch_sep_floor<D>(ctx, L)) return st;
  k_resolve<D><<<nb, BLOCK, 0, ctx->stream>>>(L, ctx->raw, ctx->eff, ctx->cnt);
  CKL();
  k_scan<<<1, BLOCK, 0, ctx->stream>>>(L.n, ctx->cnt, ctx->off);
  CKL();
  return AVS_OK;
}

template <int D>
avs_status launch_scatter(avs_ctx* ctx) {
  const Leaves L = ctx->leaves(ctx->lcur);
  const int t = ctx->lcur ^ 1;
  ProfScope ps(ctx, K_FLAGS);
  k_scatter<D><<<(L.n + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(L, ctx->eff, ctx->off, (int)ctx->cap, ctx->lt[t].level,
                                                                   ctx->lt[t].idx, ctx->pkind, ctx->psrc, ctx->pchild);
  CKL();
  return launch_leaf_geom<D>(ctx, t);
}

template <int D, typename T>
avs_status launch_remap(avs_ctx* ctx, int correction) {
  if (correction >= 3) {
    // Equilibrium bypass: the new leaves take g_eq(W) (closed onto W for 4);
    // the old distribution is not read.
    ProfScope ps(ctx, K_REMAP_CORRECT);
    ctx->lcur ^= 1;
    ctx->cur ^= 1;
    avs_status st = launch_init_vdf<D, T>(ctx, correction == 4);
    ctx->lcur ^= 1;
    ctx->cur ^= 1;
    return st;
  }
  const Leaves Lo = ctx->leaves(ctx->lcur);
  const Leaves Ln = ctx->leaves(ctx->lcur ^ 1);
  T* vout = (T*)ctx->vdf[ctx->cur ^ 1];
  {
    ProfScope ps(ctx, K_REMAP_GATHER);
    k_remap_gather<D, T><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->geo, Lo, Ln, ctx->pkind, ctx->psrc,
                                                            (const T*)ctx->vdf[ctx->cur], vout, ctx->momp);
    CKL();
  }
  if (correction > 0) {
    // the correction also leaves the moments and heat flux of the new state
    // (remap_leaves_moments)
    ProfScope ps(ctx, K_REMAP_CORRECT);
    k_remap_correct<D, T><<<ctx->nc, BLOCK, (size_t)2 * D * ctx->vg.numax * sizeof(double), ctx->stream>>>(
        ctx->geo, Ln, ctx->vg, ctx->gas, correction, ctx->W, ctx->momp, vout, ctx->bad, ctx->mom, ctx->q);
    CKL();
  }
  return AVS_OK;
}

// Corrections 1 and 2 form the moments of the new state in the correction
// kernel; the others need the moments pass after the remap.
inline bool remap_leaves_moments(int correction) { return correction == 1 || correction == 2; }

// Dynamic LDS of the sweep and remap kernels beyond the default 64 KiB (up
// to kLdsMax per workgroup on gfx950): the per-axis Maxwellian tables grow
// with the finest velocity grid.  Set once per kernel instantiation.
constexpr size_t kLdsMax = 160 * 1024 - 16 * 1024;   // room for the kernels' static LDS

template <int D, typename T>
hipError_t raise_lds() {
  static bool done = false;
  if (done) return hipSuccess;
  const int b = (int)kLdsMax;
  const void* fns[] = {(const void*)k_passC<D, T>,        (const void*)k_passC_res<D, T>,
                       (const void*)kb_passC<D, T, true>, (const void*)kb_passC<D, T, false>,
                       (const void*)k_face_eq<D, T>,      (const void*)kb_face_eq<D, T>,
                       (const void*)k_target<D, T>,       (const void*)kb_target<D, T>,
                       (const void*)k_remap_correct<D, T>, (const void*)kb_remap_correct<D, T>,
                       (const void*)k_init_vdf<D, T>};
  for (const void* fn : fns) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
  }
  done = true;
  return hipSuccess;
}

// Dispatch on (dimension, storage type).
#define DISPATCH(ctx, FN, ...)                                                       \
  ((ctx)->D == 2 ? ((ctx)->prec == AVS_FP64 ? FN<2, double>(__VA_ARGS__) : FN<2, float>(__VA_ARGS__)) \
                 : ((ctx)->prec == AVS_FP64 ? FN<3, double>(__VA_ARGS__) : FN<3, float>(__VA_ARGS__)))
#define DISPATCH_D(ctx, FN, ...) ((ctx)->D == 2 ? FN<2>(__VA_ARGS__) : FN<3>(__VA_ARGS__))

avs_status check_bad(avs_ctx* ctx) {
  int bad = INT_MAX;
  CK(hipMemcpyAsync(&bad, ctx->bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  if (bad != INT_MAX) {
    ctx->failed = true;
    if (bad < ctx->nc) return fail(AVS_E_NUMERIC, "non-physical state or singular moment system in cell %d", bad);
    return fail(AVS_E_NUMERIC, "non-physical interface state at face %d", bad - ctx->nc);
  }
  return AVS_OK;
}

avs_status upload_leaves(avs_ctx* ctx, int t, int n, const int* level, const int* idx_nd /*[n][D]*/) {
  ++ctx->leaf_gen;
  std::vector<int> ix((size_t)ctx->D * ctx->cap, 0);
  for (int k = 0; k < n; ++k)
    for (int d = 0; d < ctx->D; ++d) ix[(size_t)d * ctx->cap + k] = idx_nd[(size_t)k * ctx->D + d];
  CK(hipMemcpyAsync(ctx->lt[t].level, level, sizeof(int) * n, hipMemcpyHostToDevice, ctx->stream));
  CK(hipMemcpyAsync(ctx->lt[t].idx, ix.data(), sizeof(int) * ix.size(), hipMemcpyHostToDevice, ctx->stream));
  ctx->nleaf[t] = n;
  ctx->ld[t] = (int)round_up(n, 64);
  avs_status st = DISPATCH_D(ctx, launch_leaf_geom, ctx, t);
  if (st) return st;
  CK(hipStreamSynchronize(ctx->stream));
  return AVS_OK;
}

avs_status guard(avs_ctx* ctx) {
  if (!ctx) return fail(AVS_E_INVALID, "null context");
  if (ctx->failed) return fail(AVS_E_STATE, "context is in the failed state after an earlier device or numeric error");
  return AVS_OK;
}

}  // namespace


// ------------------------------------------------------------ batched form
struct avs_batch {
  std::vector<avs_ctx*> cases;
  int D = 2, prec = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  int chunk[4] = {CHUNK, CHUNK, CHUNK, CHUNK};   // pass-A leaves per workgroup, per leaf-count bucket
  int passc_two = -1;                           // pass C with two leaves in flight (1), one (0), default (-1)
  int nblk[BK_N] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_steps = -1;
  int graph_nblk[BK_N] = {};   // compared only once a graph exists
  int graph_chunk[4] = {-1, -1, -1, -1};
  int graph_passc = -2;
  std::vector<char> host_args;
  std::vector<char> host_remap;   // records of the batched remap
  // side streams (default priority) for the per-case adaptation and remap
  // kernels: small cases' launches run side by side instead of one after
  // another; joined back to `stream` with events
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_ev;   // [0, side.size()): joins; last: the fork
  ~avs_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : side_ev) (void)hipEventDestroy(e);
    for (hipStream_t q : side) (void)hipStreamDestroy(q);
  }
};

namespace {

// Leaf-count bucket of a case for the pass-A tile choice.
int leaf_bucket(int nleaves) { return nleaves < 1024 ? 0 : nleaves < 4096 ? 1 : nleaves < 16384 ? 2 : 3; }

size_t batch_args_bytes(int ncase) { return (size_t)round_up(2 * (size_t)ncase * sizeof(CaseArgs<double>), 256); }
size_t batch_offs_bytes(int ncase) { return (size_t)round_up(sizeof(int) * BK_N * (ncase + 1), 256); }
size_t remap_args_bytes(int ncase) { return (size_t)round_up((size_t)ncase * sizeof(RemapArgs<double>), 256); }
size_t remap_offs_bytes(int ncase) { return (size_t)round_up(sizeof(int) * BR_N * (ncase + 1), 256); }

template <typename T>
CaseArgs<T> case_args(avs_ctx* c, int flip, int chunk) {
  CaseArgs<T> a;
  a.g = c->geo;
  a.L = c->leaves(c->lcur);
  a.vg = c->vg;
  a.gas = c->gas;
  a.h = c->h;
  a.dt = c->dt;
  const int cur = c->cur ^ flip;
  a.vin = (const T*)c->vdf[cur];
  a.vout = (T*)c->vdf[cur ^ 1];
  a.fv = (T*)c->fv;
  a.bden = c->bden;
  a.bfin = c->bfin;
  a.fpar = c->fpar;
  a.F = c->F;
  a.W = flip ? c->Wn : c->W;
  a.Wn = flip ? c->W : c->Wn;
  a.q = c->q;
  a.tpar = c->tpar;
  a.lam = c->lam;
  a.bcpair = c->bcpair;
  a.mom = c->mom;
  a.bad = c->bad;
  a.fmom = c->fmom;
  a.nchs = c->nchs;
  a.chunk = chunk;
  a.gx = (int)round_up(c->nc, 8);
  return a;
}

// Upload both orientations of every case and the workgroup offsets.
template <typename T>
avs_status batch_upload(avs_batch* b) {
  avs_ctx* ctx = nullptr;
  const int n = (int)b->cases.size();
  b->host_args.resize(batch_args_bytes(n) + sizeof(int) * BK_N * (n + 1));
  CaseArgs<T>* args = reinterpret_cast<CaseArgs<T>*>(b->host_args.data());
  int* off = reinterpret_cast<int*>(b->host_args.data() + batch_args_bytes(n));
  for (int k = 0; k < BK_N; ++k) off[k * (n + 1)] = 0;
  for (int i = 0; i < n; ++i) {
    avs_ctx* c = b->cases[i];
    const int ch = b->chunk[leaf_bucket(c->nleaf[c->lcur])];
    args[i] = case_args<T>(c, 0, ch);
    args[n + i] = case_args<T>(c, 1, ch);
    const int nl = c->nleaf[c->lcur];
    const int gx = (int)round_up(c->nc, 8);
    const int fb = c->D == 2 ? face_batch<2>() : face_batch<3>();
    const int cnt[BK_N] = {gx * ((nl + ch - 1) / ch), (c->nf + fb - 1) / fb, (c->nc + BLOCK - 1) / BLOCK,
                           c->nc, gx};
    for (int k = 0; k < BK_N; ++k) off[k * (n + 1) + i + 1] = off[k * (n + 1) + i] + cnt[k];
  }
  for (int k = 0; k < BK_N; ++k) b->nblk[k] = off[k * (n + 1) + n];
  CK(hipMemcpyAsync(b->ws, b->host_args.data(), b->host_args.size(), hipMemcpyHostToDevice, b->stream));
  CK(hipStreamSynchronize(b->stream));
  return AVS_OK;
}

template <int D, typename T>
avs_status batch_launch(avs_batch* b, int nsteps) {
  avs_ctx* ctx = nullptr;
  const int n = (int)b->cases.size();
  const CaseArgs<T>* args = reinterpret_cast<const CaseArgs<T>*>(b->ws);
  const int* off = reinterpret_cast<const int*>(b->ws + batch_args_bytes(n));
  int numax = 0;
  for (avs_ctx* c : b->cases) numax = std::max(numax, c->vg.numax);
  constexpr int MAXF = Cfg<D>::MAXF;
  for (int s = 0; s < nsteps; ++s) {
    const CaseArgs<T>* a = args + (s & 1) * n;
    kb_passA<D, T><<<b->nblk[BK_PASSA], passA_threads<D>(), 0, b->stream>>>(a, off + BK_PASSA * (n + 1), n);
    CKL();
    kb_face_eq<D, T><<<b->nblk[BK_FACEQ], BLOCK, (size_t)face_batch<D>() * D * numax * sizeof(T), b->stream>>>(
        a, off + BK_FACEQ * (n + 1), n);
    CKL();
    kb_macro<D, T><<<b->nblk[BK_MACRO], BLOCK, 0, b->stream>>>(a, off + BK_MACRO * (n + 1), n);
    CKL();
    kb_target<D, T><<<b->nblk[BK_TARGET], BLOCK, (size_t)D * numax * sizeof(T), b->stream>>>(a, off + BK_TARGET * (n + 1), n);
    CKL();
    const size_t shc = (size_t)(MAXF + 1) * D * numax * sizeof(T);
    const bool two = b->passc_two < 0 ? passc_two_leaves<D, T>() : b->passc_two == 1;
    if (two)
      kb_passC<D, T, true><<<b->nblk[BK_PASSC], BLOCK, shc, b->stream>>>(a, off + BK_PASSC * (n + 1), n);
    else
      kb_passC<D, T, false><<<b->nblk[BK_PASSC], BLOCK, shc, b->stream>>>(a, off + BK_PASSC * (n + 1), n);
    CKL();
  }
  return AVS_OK;
}

// One step of every case computed into the spare buffers without taking it
// (the state W, phi^n stays where it is); the heat flux and moments that
// pass C overwrites are saved in each case's implicit-predictor and remap
// scratch and put back.  Used to time tile choices on the cases' own state.
avs_status batch_dry_step(avs_batch* b) {
  avs_ctx* ctx = nullptr;
  const bool f64 = b->prec == AVS_FP64;
  for (avs_ctx* c : b->cases) {
    CK(hipMemcpyAsync(c->irhs, c->q, sizeof(double) * c->nc * c->D, hipMemcpyDeviceToDevice, b->stream));
    CK(hipMemcpyAsync(c->momp, c->mom, sizeof(double) * c->nc * (c->D + 2), hipMemcpyDeviceToDevice, b->stream));
  }
  avs_status st = f64 ? batch_upload<double>(b) : batch_upload<float>(b);
  if (st) return st;
  st = b->D == 2 ? (f64 ? batch_launch<2, double>(b, 1) : batch_launch<2, float>(b, 1))
                 : (f64 ? batch_launch<3, double>(b, 1) : batch_launch<3, float>(b, 1));
  if (st) return st;
  for (avs_ctx* c : b->cases) {
    CK(hipMemcpyAsync(c->q, c->irhs, sizeof(double) * c->nc * c->D, hipMemcpyDeviceToDevice, b->stream));
    CK(hipMemcpyAsync(c->mom, c->momp, sizeof(double) * c->nc * (c->D + 2), hipMemcpyDeviceToDevice, b->stream));
  }
  return AVS_OK;
}

avs_status batch_run(avs_batch* b, int nsteps, bool graph) {
  avs_ctx* ctx = nullptr;
  const bool f64 = b->prec == AVS_FP64;
  avs_status st = f64 ? batch_upload<double>(b) : batch_upload<float>(b);
  if (st) return st;
  if (!graph) {
    st = b->D == 2 ? (f64 ? batch_launch<2, double>(b, nsteps) : batch_launch<2, float>(b, nsteps))
                   : (f64 ? batch_launch<3, double>(b, nsteps) : batch_launch<3, float>(b, nsteps));
  } else {
    bool same = b->exec && b->graph_steps == nsteps && b->graph_passc == b->passc_two;
    for (int q = 0; q < 4; ++q) same = same && b->graph_chunk[q] == b->chunk[q];
    for (int k = 0; k < BK_N; ++k) same = same && b->graph_nblk[k] == b->nblk[k];
    if (!same) {
      if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
      if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
      CK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      st = b->D == 2 ? (f64 ? batch_launch<2, double>(b, nsteps) : batch_launch<2, float>(b, nsteps))
                     : (f64 ? batch_launch<3, double>(b, nsteps) : batch_launch<3, float>(b, nsteps));
      hipGraph_t gr = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->stream, &gr);
      if (st) { if (gr) (void)hipGraphDestroy(gr); return st; }
      CK(ec);
      b->graph = gr;
      CK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->graph_steps = nsteps;
      b->graph_passc = b->passc_two;
      for (int q = 0; q < 4; ++q) b->graph_chunk[q] = b->chunk[q];
      for (int k = 0; k < BK_N; ++k) b->graph_nblk[k] = b->nblk[k];
    }
    CK(hipGraphLaunch(b->exec, b->stream));
  }
  if (st) return st;
  // the members now hold their state in the other buffers after an odd count
  if (nsteps & 1)
    for (avs_ctx* c : b->cases) {
      std::swap(c->W, c->Wn);
      c->cur ^= 1;
    }
  return AVS_OK;
}

}  // namespace

// ------------------------------------- no-allocation totals (static scratch)
// Device memory of avs_moments_noalloc: per-block partial sums of
// sum_i V_i W_i, then the totals staged for the host copy.  One array per
// device (each GPU holds its own copy for the life of the process); every
// call on a device shares it, so calls that overlap on one device race.
constexpr int NOALLOC_CELLS_PER_BLOCK = 1024;
constexpr int NOALLOC_MAX_BLOCKS = 1024;                                   // at most 1 048 576 cells
constexpr int NOALLOC_DOUBLES = (NOALLOC_MAX_BLOCKS + 1) * (3 + 2);        // D + 2 <= 5 per partial
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};   // the array's device address, per device

// Resolve the array's address on device dev (made current for the call);
// done once per device, at context set-up.  The array's name in host code
// is a host-side stand-in, never a device address: only these pointers are
// handed to kernels.
hipError_t resolve_scratch(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    (void)hipGetLastError();     // keep the failure out of later launch checks
    return e;
  }
  g_scratch_dev[dev] = static_cast<double*>(p);
  return hipSuccess;
}

// ---------------------------------------------- automatic velocity space
// Sec. 3.5: parameters of the velocity space from the freestream.
avs_status auto_params_host(const avs_flow* f, avs_auto* p, avs_vspace* vs) {
  if (!f) return fail(AVS_E_INVALID, "null flow descriptor");
  if (f->dim != 2 && f->dim != 3) return fail(AVS_E_INVALID, "flow.dim must be 2 or 3 (got %d)", f->dim);
  auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
  if (!pos(f->R) || !(std::isfinite(f->gamma) && f->gamma > 1.0)) return fail(AVS_E_INVALID, "need R > 0 and gamma > 1");
  if (!(std::isfinite(f->Ma) && f->Ma >= 0.0)) return fail(AVS_E_INVALID, "Ma must be finite and >= 0");
  if (!pos(f->T_inf) || !pos(f->T_wall) || !pos(f->rho_inf)) return fail(AVS_E_INVALID, "T_inf, T_wall and rho_inf must be > 0");
  if (!pos(f->rdv_sigmas) || !pos(f->h_std)) return fail(AVS_E_INVALID, "rdv_sigmas and h_std must be > 0");
  const int D = f->dim;
  double e[3] = {0.0, 0.0, 0.0}, norm = 0.0;
  for (int d = 0; d < D; ++d) norm += f->direction[d] * f->direction[d];
  norm = std::sqrt(norm);
  if (f->Ma > 0.0 && !(norm > 0.0 && std::isfinite(norm))) return fail(AVS_E_INVALID, "flow.direction must be non-zero");
  if (norm > 0.0)
    for (int d = 0; d < D; ++d) e[d] = f->direction[d] / norm;
  avs_auto a{};
  a.T0 = f->T_inf * (1.0 + 0.5 * (f->gamma - 1.0) * f->Ma * f->Ma);
  a.sigma_inf = std::sqrt(f->R * f->T_inf);
  a.sigma_0 = std::sqrt(f->R * a.T0);
  a.sigma_w = std::sqrt(f->R * f->T_wall);
  a.U_inf = f->Ma * std::sqrt(f->gamma * f->R * f->T_inf);
  a.R_dv = f->rdv_sigmas * a.sigma_0;
  for (int d = 0; d < D; ++d) a.centre[d] = 0.4 * a.U_inf * e[d];
  const double span = 2.0 * a.R_dv / f->h_std;   // elements per axis needed at h_std
  int L = 0;
  while (std::ldexp(1.0, L) < span) {
    if (++L > 30) return fail(AVS_E_INVALID, "velocity box needs more than 2^30 elements per axis at h_std");
  }
  a.L_max = L;
  a.h_min = 2.0 * a.R_dv / std::ldexp(1.0, L);
  a.L_w = (f->T_wall / f->T_inf < 4.0) ? a.L_max : a.L_max - 1;
  a.L_min = (D == 2 && f->Ma > 5.0) ? 4 : 3;
  a.L_sep = std::max(a.L_min, a.L_w - 1);
  a.k_sigma = std::exp(-8.0);                   // f(4) / f(0) of the standard normal density
  a.C1 = 13.749 * std::pow(f->Ma, -1.465);      // +inf at Ma = 0: nothing splits
  a.C2 = a.k_sigma * a.C1;
  const int lr = std::min(a.L_min, a.L_max);
  const int ml = a.L_max - lr;
  if (ml > 12) return fail(AVS_E_INVALID, "velocity space needs %d levels below the roots (at most 12)", ml);
  if (p) *p = a;
  if (vs) {
    avs_vspace v{};
    v.dim = D;
    v.max_level = ml;
    for (int d = 0; d < 3; ++d) {
      v.base[d] = d < D ? (1 << lr) : 1;
      v.lo[d] = d < D ? a.centre[d] - a.R_dv : 0.0;
      v.hi[d] = d < D ? a.centre[d] + a.R_dv : 1.0;
    }
    v.leaf_capacity = std::min<int64_t>(int64_t(1) << std::min(D * a.L_max, 26), int64_t(1) << 26);
    *vs = v;
  }
  return AVS_OK;
}

extern "C" {

double avs_mu_ref_from_kn(double Kn, double omega, double R, double T_ref, double rho_ref, double L_ref) {
  return Kn * L_ref * 15.0 * rho_ref * sqrt(2.0 * M_PI * R * T_ref) / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega));
}

size_t avs_vdf_bytes(const avs_vspace* vs, const avs_pmesh* pm, const avs_opts* op) {
  if (check_args(vs, pm, op)) return 0;
  avs_ctx x;
  fill_dims(x, vs, pm, op);
  return (2 * (size_t)x.nc + (size_t)std::max(x.nf, 1)) * x.P * x.cap * x.esize();
}

size_t avs_workspace_bytes(const avs_vspace* vs, const avs_pmesh* pm, const avs_opts* op) {
  if (check_args(vs, pm, op)) return 0;
  avs_ctx x;
  fill_dims(x, vs, pm, op);
  Carver c{nullptr};
  carve(x, c);
  return round_up((int64_t)c.off, 256);
}

avs_status avs_init_mesh(const avs_vspace* vs, const avs_pmesh* pm, const avs_gas* gas, const avs_opts* op,
                         const double* prim0_host, void* vdf_dev, size_t vdf_bytes, void* workspace_dev,
                         size_t workspace_bytes, void* hip_stream, avs_ctx** out) {
  avs_ctx* ctx = nullptr;
  if (!out) return fail(AVS_E_INVALID, "out is null");
  *out = nullptr;
  if (avs_status st = check_args(vs, pm, op)) return st;
  if (!gas || !prim0_host || !vdf_dev || !workspace_dev) return fail(AVS_E_INVALID, "null gas/prim0/vdf/workspace pointer");
  if (!(gas->R > 0 && gas->mu_ref > 0 && gas->T_ref > 0 && gas->Pr > 0) || (gas->model != 0 && gas->model != 1))
    return fail(AVS_E_INVALID, "invalid gas parameters");
  if ((gas->law != 0 && gas->law != 1) || !(gas->C_s >= 0.0 && std::isfinite(gas->C_s)))
    return fail(AVS_E_INVALID, "viscosity law must be 0 (power) or 1 (Sutherland, C_s >= 0)");
  if (vdf_bytes < avs_vdf_bytes(vs, pm, op)) return fail(AVS_E_INVALID, "vdf region too small (%zu < %zu)", vdf_bytes, avs_vdf_bytes(vs, pm, op));
  if (workspace_bytes < avs_workspace_bytes(vs, pm, op))
    return fail(AVS_E_INVALID, "workspace too small (%zu < %zu)", workspace_bytes, avs_workspace_bytes(vs, pm, op));
  if (((uintptr_t)vdf_dev & 255) || ((uintptr_t)workspace_dev & 255)) return fail(AVS_E_INVALID, "device regions must be 256-byte aligned");
  const int D = vs->dim, N = D + 2;
  const int64_t nc = pm->ncells, nf = pm->nfaces;
  if (!pm->cell_vol || !pm->cell_ctr || (nf > 0 && (!pm->face_lr || !pm->face_area || !pm->face_nrm || !pm->face_ctr)))
    return fail(AVS_E_INVALID, "null mesh array");
  if (pm->nbc < 0 || (pm->nbc > 0 && (!pm->bc_kind || !pm->bc_state))) return fail(AVS_E_INVALID, "invalid bc arrays");
  const int maxf = D == 2 ? MAXF2 : MAXF3;
  // ---- validate mesh and build per-cell slot tables (host)
  std::vector<int> nslot(nc, 0), s_face(nc * maxf, 0), s_nbr(nc * maxf, -1);
  std::vector<double> s_sig(nc * maxf, 0.0), s_sigA(nc * maxf, 0.0), s_d(nc * maxf * D, 0.0), s_dx(nc * maxf * D, 0.0),
      s_lsq(nc * maxf * D, 0.0);
  std::vector<int> f_L(nf + 1, 0), f_R(nf + 1, 0), f_sL(nf + 1, 0), f_sR(nf + 1, 0), f_int, f_bnd;
  std::vector<double> f_nrm((nf + 1) * D, 0.0);
  for (int64_t i = 0; i < nc; ++i)
    if (!(pm->cell_vol[i] > 0)) return fail(AVS_E_INVALID, "cell %" PRId64 " has non-positive volume", i);
  for (int b = 0; b < pm->nbc; ++b)
    if (pm->bc_kind[b] != AVS_BC_WALL && pm->bc_kind[b] != AVS_BC_FARFIELD) return fail(AVS_E_INVALID, "bc %d: unknown kind", b);
  for (int64_t f = 0; f < nf; ++f) {
    const int64_t L = pm->face_lr[2 * f], R = pm->face_lr[2 * f + 1];
    if (L < 0 || L >= nc) return fail(AVS_E_INVALID, "face %" PRId64 ": L out of range", f);
    if (R >= nc || (R < 0 && -1 - R >= pm->nbc)) return fail(AVS_E_INVALID, "face %" PRId64 ": R out of range", f);
    if (!(pm->face_area[f] >= 0)) return fail(AVS_E_INVALID, "face %" PRId64 ": negative area", f);
    const double* xf = pm->face_ctr + f * D;
    double xR[3] = {0, 0, 0};
    if (R >= 0)
      for (int d = 0; d < D; ++d) xR[d] = pm->cell_ctr[R * D + d] + (pm->face_shift ? pm->face_shift[f * D + d] : 0.0);
    if (nslot[L] >= maxf) return fail(AVS_E_INVALID, "cell %" PRId64 " has more than %d faces", L, maxf);
    int s = nslot[L]++;
    s_face[L * maxf + s] = (int)f;
    s_nbr[L * maxf + s] = R >= 0 ? (int)R : -1;
    s_sig[L * maxf + s] = 1.0;
    s_sigA[L * maxf + s] = pm->face_area[f];
    for (int d = 0; d < D; ++d) {
      s_d[(L * maxf + s) * D + d] = xf[d] - pm->cell_ctr[L * D + d];
      if (R >= 0) s_dx[(L * maxf + s) * D + d] = xR[d] - pm->cell_ctr[L * D + d];
    }
    f_L[f] = (int)L;
    f_R[f] = (int)R;
    f_sL[f] = s;
    for (int d = 0; d < D; ++d) f_nrm[f * D + d] = pm->face_nrm[f * D + d];
    if (R >= 0) {
      if (nslot[R] >= maxf) return fail(AVS_E_INVALID, "cell %" PRId64 " has more than %d faces", R, maxf);
      s = nslot[R]++;
      s_face[R * maxf + s] = (int)f;
      s_nbr[R * maxf + s] = (int)L;
      s_sig[R * maxf + s] = -1.0;
      s_sigA[R * maxf + s] = -pm->face_area[f];
      for (int d = 0; d < D; ++d) {
        s_d[(R * maxf + s) * D + d] = xf[d] - xR[d];
        s_dx[(R * maxf + s) * D + d] = pm->cell_ctr[L * D + d] - xR[d];
      }
      f_sR[f] = s;
      f_int.push_back((int)f);
    } else {
      f_bnd.push_back((int)f);
    }
  }
  std::vector<double> eps2(nc), dtv(nc);
  for (int64_t i = 0; i < nc; ++i) {
    double M[9] = {0}, Mi[9];
    for (int s = 0; s < nslot[i]; ++s) {
      if (s_nbr[i * maxf + s] < 0) continue;
      const double* dx = &s_dx[(i * maxf + s) * D];
      double r2 = 0.0;
      for (int d = 0; d < D; ++d) r2 += dx[d] * dx[d];
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) M[a * D + b] += dx[a] * dx[b] / r2;
    }
    pinv_sym(D, M, Mi);
    for (int s = 0; s < nslot[i]; ++s) {
      if (s_nbr[i * maxf + s] < 0) continue;
      const double* dx = &s_dx[(i * maxf + s) * D];
      double r2 = 0.0;
      for (int d = 0; d < D; ++d) r2 += dx[d] * dx[d];
      for (int a = 0; a < D; ++a) {
        double v = 0.0;
        for (int b = 0; b < D; ++b) v += Mi[a * D + b] * dx[b] / r2;
        s_lsq[(i * maxf + s) * D + a] = v;
      }
    }
    eps2[i] = pow(op->venkat_K * pow(pm->cell_vol[i], 1.0 / D), 3.0);
    dtv[i] = op->dt / pm->cell_vol[i];
  }
  // Half step of the interface VDF: dt/2, capped at half of the step at
  // which some cell's outflow over the whole velocity box equals its
  // content (min_i V_i / (1/2 sum_f A_f sum_d |n_fd| X_d), X_d = max(|lo_d|,
  // |hi_d|)), so that x_f - xi h stays within reach of the upwind cell when
  // an implicit step is longer than the explicit bound (Sec. 2.3.3).
  double hcap = INFINITY;
  for (int64_t i = 0; i < nc; ++i) {
    double out = 0.0;
    for (int s = 0; s < nslot[i]; ++s) {
      const int f = s_face[i * maxf + s];
      double nx = 0.0;
      for (int d = 0; d < D; ++d) nx += fabs(pm->face_nrm[(size_t)f * D + d]) * std::max(fabs(vs->lo[d]), fabs(vs->hi[d]));
      out += 0.5 * pm->face_area[f] * nx;
    }
    if (out > 0.0) hcap = std::min(hcap, pm->cell_vol[i] / out);
  }
  const double h_flux = std::min(0.5 * op->dt, 0.5 * hcap);
  // greedy colouring of the face-neighbour graph in cell order (each cell
  // takes the smallest colour no lower-numbered neighbour holds); the cells
  // of one colour share no face, so a Gauss-Seidel sweep updates a colour at once
  std::vector<int> colour(nc, 0), col_cells;
  int ncol = 0;
  for (int64_t i = 0; i < nc; ++i) {
    unsigned used = 0;
    for (int s = 0; s < nslot[i]; ++s) {
      const int j = s_nbr[i * maxf + s];
      if (j >= 0 && j < i) used |= 1u << colour[j];
    }
    int c = 0;
    while (used & (1u << c)) ++c;
    colour[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  std::vector<int> col_off(ncol + 1, 0);
  for (int64_t i = 0; i < nc; ++i) ++col_off[colour[i] + 1];
  for (int c = 0; c < ncol; ++c) col_off[c + 1] += col_off[c];
  col_cells.resize(nc);
  {
    std::vector<int> fillp(col_off.begin(), col_off.end() - 1);
    for (int64_t i = 0; i < nc; ++i) col_cells[fillp[colour[i]]++] = (int)i;
  }
  // locality order: Morton key of the centres quantised on 2^(60/D) steps per axis
  std::vector<int> order(nc);
  {
    double lo_[3] = {1e300, 1e300, 1e300}, hi_[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < nc; ++i)
      for (int d = 0; d < D; ++d) {
        lo_[d] = std::min(lo_[d], pm->cell_ctr[i * D + d]);
        hi_[d] = std::max(hi_[d], pm->cell_ctr[i * D + d]);
      }
    const int bits = 60 / D;
    std::vector<std::pair<uint64_t, int>> key(nc);
    for (int64_t i = 0; i < nc; ++i) {
      uint64_t q[3] = {0, 0, 0}, kk = 0;
      for (int d = 0; d < D; ++d) {
        const double span = hi_[d] > lo_[d] ? hi_[d] - lo_[d] : 1.0;
        q[d] = (uint64_t)std::min((double)((1ull << bits) - 1), (pm->cell_ctr[i * D + d] - lo_[d]) / span * (double)(1ull << bits));
      }
      for (int b = 0; b < bits; ++b)
        for (int d = 0; d < D; ++d) kk |= ((q[d] >> b) & 1ull) << (D * b + d);
      key[i] = {kk, (int)i};
    }
    std::sort(key.begin(), key.end());
    for (int64_t i = 0; i < nc; ++i) order[i] = key[i].second;
  }
  std::vector<double> W0(nc * N);
  for (int64_t i = 0; i < nc; ++i) {
    const double* pr = prim0_host + i * N;
    if (!(pr[0] > 0 && pr[1 + D] > 0)) return fail(AVS_E_INVALID, "initial state of cell %" PRId64 " is not physical", i);
    conserved_host(D, gas->R, pr, &W0[i * N]);
  }
  // ---- device: everything above is host work on the caller's arrays
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(AVS_E_HIP, "hipGetDevice failed");
  // the no-allocation entry point's array on this device: a failure here only
  // disables that entry point (it reports it), the context is unaffected
  (void)resolve_scratch(device);
  // ---- context
  ctx = new avs_ctx();
  avs_ctx& x = *ctx;
  fill_dims(x, vs, pm, op);
  x.n_int = (int)f_int.size();
  x.n_bnd = (int)f_bnd.size();
  x.lmax = vs->max_level;
  for (int d = 0; d < 3; ++d) {
    x.base[d] = d < D ? vs->base[d] : 1;
    x.lo[d] = d < D ? vs->lo[d] : 0.0;
    x.hi[d] = d < D ? vs->hi[d] : 1.0;
    x.vg.nu[d] = d < D ? vs->base[d] << (vs->max_level + 1) : 1;
    x.vg.x0[d] = x.lo[d];
    x.vg.hh[d] = (x.hi[d] - x.lo[d]) / (double)((int64_t)x.base[d] << (vs->max_level + 1));
  }
  x.vg.numax = numax_of(vs);
  x.gas = GasP{gas->R, gas->Pr, gas->omega, gas->mu_ref, gas->T_ref, gas->model, gas->law, gas->C_s};
  x.dt = op->dt;
  x.h = h_flux;
  x.Kv = op->venkat_K;
  x.stream = (hipStream_t)hip_stream;
  x.device = device;
  x.vol_host.assign(pm->cell_vol, pm->cell_vol + nc);
  x.vdf_buf_bytes = (size_t)x.P * x.nc * x.cap * x.esize();
  x.vdf[0] = vdf_dev;
  x.vdf[1] = (char*)vdf_dev + x.vdf_buf_bytes;
  x.fv = (char*)vdf_dev + 2 * x.vdf_buf_bytes;
  Carver cv{(char*)workspace_dev};
  carve(x, cv);
  const int P = x.P;
  // LDS budget of the sweep kernels (pass C holds MAXF + 1 tables of D rows,
  // the face equilibrium one per face of its batch)
  const int ntab = std::max(x.maxf + 1, D == 2 ? face_batch<2>() : face_batch<3>());
  const size_t lds_need = (size_t)ntab * D * x.vg.numax * x.esize();
  if (lds_need > kLdsMax) {
    delete ctx;
    return fail(AVS_E_INVALID, "velocity grid too fine for the LDS tables (2 base 2^max_level = %d needs %zu B > %zu B)",
                x.vg.numax, lds_need, kLdsMax);
  }
  if (lds_need + 8192 > 64 * 1024) {
    const hipError_t e = D == 2 ? (x.prec == AVS_FP64 ? raise_lds<2, double>() : raise_lds<2, float>())
                                : (x.prec == AVS_FP64 ? raise_lds<3, double>() : raise_lds<3, float>());
    if (e != hipSuccess) {
      delete ctx;
      return fail(AVS_E_HIP, "hipFuncSetAttribute (dynamic LDS %zu B): %s", kLdsMax, hipGetErrorString(e));
    }
  }
  auto H2D = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, x.stream);
  };
  std::vector<int> kinds(pm->bc_kind, pm->bc_kind + pm->nbc);
  std::vector<double> bprim(pm->bc_state, pm->bc_state + (size_t)pm->nbc * N);
  int badinit[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
#define CKI(e)                                  \
  do {                                          \
    hipError_t er_ = (e);                       \
    if (er_ != hipSuccess) {                    \
      delete ctx;                               \
      return fail(AVS_E_HIP, "%s: %s", #e, hipGetErrorString(er_)); \
    }                                           \
  } while (0)
  CKI(H2D((void*)x.geo.order, order.data(), sizeof(int) * nc));
  CKI(H2D((void*)x.geo.vol, pm->cell_vol, sizeof(double) * nc));
  CKI(H2D((void*)x.geo.eps2, eps2.data(), sizeof(double) * nc));
  CKI(H2D((void*)x.geo.dtv, dtv.data(), sizeof(double) * nc));
  CKI(H2D((void*)x.geo.nslot, nslot.data(), sizeof(int) * nc));
  CKI(H2D((void*)x.geo.s_face, s_face.data(), sizeof(int) * s_face.size()));
  CKI(H2D((void*)x.geo.s_nbr, s_nbr.data(), sizeof(int) * s_nbr.size()));
  CKI(H2D((void*)x.geo.s_sig, s_sig.data(), sizeof(double) * s_sig.size()));
  CKI(H2D((void*)x.geo.s_sigA, s_sigA.data(), sizeof(double) * s_sigA.size()));
  CKI(H2D((void*)x.geo.s_d, s_d.data(), sizeof(double) * s_d.size()));
  CKI(H2D((void*)x.geo.s_dx, s_dx.data(), sizeof(double) * s_dx.size()));
  CKI(H2D((void*)x.geo.s_lsq, s_lsq.data(), sizeof(double) * s_lsq.size()));
  CKI(H2D((void*)x.geo.f_L, f_L.data(), sizeof(int) * f_L.size()));
  CKI(H2D((void*)x.geo.f_R, f_R.data(), sizeof(int) * f_R.size()));
  CKI(H2D((void*)x.geo.f_sL, f_sL.data(), sizeof(int) * f_sL.size()));
  CKI(H2D((void*)x.geo.f_sR, f_sR.data(), sizeof(int) * f_sR.size()));
  CKI(H2D((void*)x.geo.f_nrm, f_nrm.data(), sizeof(double) * f_nrm.size()));
  if (!f_int.empty()) CKI(H2D((void*)x.geo.f_int, f_int.data(), sizeof(int) * f_int.size()));
  if (!f_bnd.empty()) CKI(H2D((void*)x.geo.f_bnd, f_bnd.data(), sizeof(int) * f_bnd.size()));
  if (pm->nbc > 0) {
    CKI(H2D((void*)x.geo.bc_kind, kinds.data(), sizeof(int) * kinds.size()));
    CKI(H2D((void*)x.geo.bc_prim, bprim.data(), sizeof(double) * bprim.size()));
  }
  CKI(H2D(x.W, W0.data(), sizeof(double) * W0.size()));
  CKI(H2D(x.bad, badinit, sizeof badinit));
  CKI(H2D(x.col_cells, col_cells.data(), sizeof(int) * nc));
  x.col_off = col_off;
  x.geo.D = D;
  x.geo.P = P;
  x.geo.nc = (int)nc;
  x.geo.nf = (int)nf;
  x.geo.maxf = maxf;
  x.geo.nbc = pm->nbc;
  x.geo.n_int = x.n_int;
  x.geo.n_bnd = x.n_bnd;
  // ---- level-0 forest in depth-first order
  std::vector<std::pair<uint64_t, std::vector<int>>> roots;
  const int b0 = x.base[0], b1 = x.base[1], b2 = D == 3 ? x.base[2] : 1;
  for (int c = 0; c < b2; ++c)
    for (int b = 0; b < b1; ++b)
      for (int a = 0; a < b0; ++a) {
        std::vector<int> ix = {a, b, c};
        ix.resize(D);
        roots.push_back({morton(D, x.lmax, 0, ix.data()), ix});
      }
  std::sort(roots.begin(), roots.end(), [](const auto& p, const auto& q) { return p.first < q.first; });
  std::vector<int> lev(roots.size(), 0), idx(roots.size() * D);
  for (size_t k = 0; k < roots.size(); ++k)
    for (int d = 0; d < D; ++d) idx[k * D + d] = roots[k].second[d];
  if (avs_status st = upload_leaves(ctx, 0, (int)roots.size(), lev.data(), idx.data())) { delete ctx; return st; }
  x.lcur = 0;
  x.cur = 0;
  avs_status st = DISPATCH(ctx, launch_init_vdf, ctx);
  if (!st) st = DISPATCH(ctx, launch_moments, ctx);
  if (!st) st = DISPATCH_D(ctx, launch_bc_tables, ctx);
  if (!st) st = check_bad(ctx);
  if (st) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return AVS_OK;
}

avs_status avs_step(avs_ctx* ctx, int32_t nsteps, double* residual_host) {
  if (avs_status st = guard(ctx)) return st;
  if (nsteps < 0) return fail(AVS_E_INVALID, "nsteps < 0");
  for (int n = 0; n < nsteps; ++n) {
    const bool last = residual_host && n == nsteps - 1;
    if (avs_status st = DISPATCH(ctx, launch_step, ctx, last)) return st;
  }
  if (residual_host) {
    if (nsteps == 0) return fail(AVS_E_INVALID, "residual requested for zero steps");
    CK(hipMemcpyAsync(residual_host, ctx->res, sizeof(double) * (ctx->D + 2), hipMemcpyDeviceToHost, ctx->stream));
    if (avs_status st = check_bad(ctx)) return st;
  }
  return AVS_OK;
}

avs_status avs_check(avs_ctx* ctx) {
  if (avs_status st = guard(ctx)) return st;
  return check_bad(ctx);
}

avs_status avs_implicit_bytes(const avs_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return fail(AVS_E_INVALID, "null argument");
  *bytes = ctx->vdf_buf_bytes;
  return AVS_OK;
}

avs_status avs_step_implicit(avs_ctx* ctx, int32_t nsteps, int32_t macro_sweeps, int32_t micro_sweeps, void* res_dev,
                             size_t res_bytes, double* residual_host) {
  if (avs_status st = guard(ctx)) return st;
  if (nsteps < 0 || macro_sweeps < 0 || micro_sweeps < 0) return fail(AVS_E_INVALID, "negative step or sweep count");
  if (!res_dev || ((uintptr_t)res_dev & 255)) return fail(AVS_E_INVALID, "res_dev must be a 256-byte aligned device region");
  if (res_bytes < ctx->vdf_buf_bytes)
    return fail(AVS_E_INVALID, "res region too small (%zu < %zu)", res_bytes, ctx->vdf_buf_bytes);
  for (int n = 0; n < nsteps; ++n) {
    const bool last = residual_host && n == nsteps - 1;
    avs_status st = ctx->D == 2
                        ? (ctx->prec == AVS_FP64 ? launch_step_implicit<2, double>(ctx, macro_sweeps, micro_sweeps, (double*)res_dev, last)
                                                 : launch_step_implicit<2, float>(ctx, macro_sweeps, micro_sweeps, (float*)res_dev, last))
                        : (ctx->prec == AVS_FP64 ? launch_step_implicit<3, double>(ctx, macro_sweeps, micro_sweeps, (double*)res_dev, last)
                                                 : launch_step_implicit<3, float>(ctx, macro_sweeps, micro_sweeps, (float*)res_dev, last));
    if (st) return st;
  }
  if (residual_host) {
    if (nsteps == 0) return fail(AVS_E_INVALID, "residual requested for zero steps");
    CK(hipMemcpyAsync(residual_host, ctx->res, sizeof(double) * (ctx->D + 2), hipMemcpyDeviceToHost, ctx->stream));
  }
  return check_bad(ctx);
}

avs_status avs_rykov_equilibrium(avs_ctx* ctx, const avs_rykov* gas, const double* states_dev, int64_t n, void* out_dev,
                                 size_t out_bytes) {
  if (avs_status st = guard(ctx)) return st;
  if (!gas || !states_dev || !out_dev) return fail(AVS_E_INVALID, "null argument");
  if (n < 0 || n > INT_MAX) return fail(AVS_E_INVALID, "n out of range");
  if (!(gas->Z_rot >= 1.0 && std::isfinite(gas->Z_rot)) || !(gas->delta > 0.0 && gas->delta <= 1.0) ||
      !std::isfinite(gas->omega0) || !std::isfinite(gas->omega1))
    return fail(AVS_E_INVALID, "Rykov parameters: Z_rot >= 1, 0 < delta <= 1, finite omega_0 and omega_1");
  const int ld = ctx->ld[ctx->lcur];
  const size_t need = (size_t)3 * (size_t)n * ld * ctx->esize();
  if (out_bytes < need) return fail(AVS_E_INVALID, "out region too small (%zu < %zu)", out_bytes, need);
  if (n == 0) return AVS_OK;
  const Leaves L = ctx->leaves(ctx->lcur);
  const RykovP gp{ctx->gas.R, gas->Z_rot, gas->delta, gas->omega0, gas->omega1};
  const size_t shm = (size_t)2 * ctx->D * ctx->vg.numax * sizeof(double);
  if (shm > 60 * 1024) return fail(AVS_E_INVALID, "velocity grid too fine for the equilibrium tables");
  if (ctx->D == 2) {
    if (ctx->prec == AVS_FP64) k_rykov_eq<2, double><<<(unsigned)n, BLOCK, shm, ctx->stream>>>(L, ctx->vg, gp, (int)n, states_dev, (double*)out_dev);
    else k_rykov_eq<2, float><<<(unsigned)n, BLOCK, shm, ctx->stream>>>(L, ctx->vg, gp, (int)n, states_dev, (float*)out_dev);
  } else {
    if (ctx->prec == AVS_FP64) k_rykov_eq<3, double><<<(unsigned)n, BLOCK, shm, ctx->stream>>>(L, ctx->vg, gp, (int)n, states_dev, (double*)out_dev);
    else k_rykov_eq<3, float><<<(unsigned)n, BLOCK, shm, ctx->stream>>>(L, ctx->vg, gp, (int)n, states_dev, (float*)out_dev);
  }
  CKL();
  return AVS_OK;
}

// ------------------------------------------------ diatomic (Rykov) path
static avs_status finish_plan(avs_ctx* ctx, int8_t* flags_dev, int64_t* n_new_host, bool* capacity_ok);
static avs_status upload_probes(avs_ctx* ctx, const double* probes_host, int32_t nprobes, bool diatomic = false);

struct avs_dia {
  avs_ctx* ctx = nullptr;
  DiaGas gp{};
  double *v[2] = {nullptr, nullptr}, *fv = nullptr, *W[2] = {nullptr, nullptr};
  double *q = nullptr, *F = nullptr, *tp = nullptr, *lam = nullptr;
  double *rf = nullptr, *irhs = nullptr, *idiag = nullptr, *dW = nullptr;   // implicit predictor
  int* bad = nullptr;
  int cur = 0;
  int64_t gen = 0;
  int64_t max_leaves = 0;
};

}  // extern "C"

namespace {
size_t dia_layout(const avs_ctx* c, int64_t max_leaves, avs_dia* d, char* base) {
  Carver cv{base};
  // rows for at most max_leaves leaves
  const size_t nc = c->nc, nf = c->nf, cap = (size_t)round_up(max_leaves, 64);
  const size_t D = c->D, NW = D + 3, NQ = 2 * D, NT = 6 + 3 * D;
  for (int t = 0; t < 2; ++t) {
    double* p = cv.take<double>(3 * nc * cap);
    if (d) d->v[t] = p;
  }
  double* fv = cv.take<double>(3 * (nf + 1) * cap);
  double* W0 = cv.take<double>(nc * NW);
  double* W1 = cv.take<double>(nc * NW);
  double* q = cv.take<double>(nc * NQ);
  double* F = cv.take<double>((nf + 1) * NW);
  double* tp = cv.take<double>(nc * NT);
  double* lam = cv.take<double>(nc * NW);
  double* rf = cv.take<double>(nf + 1);
  double* irhs = cv.take<double>(nc * NW);
  double* idiag = cv.take<double>(nc);
  double* dW = cv.take<double>(nc * NW);
  int* bad = cv.take<int>(4);
  if (d) {
    d->fv = fv; d->W[0] = W0; d->W[1] = W1; d->q = q; d->F = F; d->tp = tp; d->lam = lam; d->bad = bad;
    d->rf = rf; d->irhs = irhs; d->idiag = idiag; d->dW = dW;
  }
  return cv.off;
}

avs_status dia_check_bad(avs_dia* d) {
  avs_ctx* ctx = d->ctx;
  int bad = INT_MAX;
  CK(hipMemcpyAsync(&bad, d->bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  if (bad != INT_MAX) return fail(AVS_E_NUMERIC, "diatomic path: non-physical state or singular closure at %d", bad);
  return AVS_OK;
}

size_t dia_shm(const avs_ctx* ctx) { return (size_t)2 * ctx->D * ctx->vg.numax * sizeof(double); }

template <int D>
avs_status dia_init(avs_dia* d) {
  avs_ctx* ctx = d->ctx;
  const Leaves L = ctx->leaves(ctx->lcur);
  const int nc = ctx->nc;
  const unsigned gc = (unsigned)((nc + BLOCK - 1) / BLOCK);
  k_dg_initrec<D><<<gc, BLOCK, 0, ctx->stream>>>(nc, d->gp, d->W[0], d->tp, d->bad);
  CKL();
  k_dg_target<D><<<nc, BLOCK, dia_shm(ctx), ctx->stream>>>(ctx->geo, L, ctx->vg, d->gp, d->tp, d->W[0], d->lam, 1,
                                                           d->bad);
  CKL();
  k_dg_update<D><<<nc, BLOCK, dia_shm(ctx), ctx->stream>>>(ctx->geo, L, ctx->vg, d->gp, nullptr, nullptr, d->v[0], d->tp,
                                                           d->lam, d->q, 1);
  CKL();
  return AVS_OK;
}

template <int D>
avs_status dia_steps(avs_dia* d, int nsteps) {
  avs_ctx* ctx = d->ctx;
  const Leaves L = ctx->leaves(ctx->lcur);
  const unsigned gc = (unsigned)((ctx->nc + BLOCK - 1) / BLOCK);
  const size_t shm = dia_shm(ctx);
  for (int s = 0; s < nsteps; ++s) {
    const int c = d->cur;
    k_dg_recon<D><<<dim3((unsigned)round_up(ctx->nc, 8), (unsigned)((L.n + CHUNK - 1) / CHUNK)), BLOCK, 0,
                    ctx->stream>>>(ctx->geo, L, ctx->h, d->v[c], d->fv, d->gp, CHUNK);
    CKL();
    k_dg_face<D><<<ctx->nf, BLOCK, shm, ctx->stream>>>(ctx->geo, L, ctx->vg, ctx->gas, d->gp, ctx->h, d->fv, d->F,
                                                       d->bad, nullptr, nullptr);
    CKL();
    k_dg_macro<D><<<gc, BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->gas, d->gp, ctx->dt, d->F, d->W[c], d->W[c ^ 1], d->q,
                                                 d->tp, d->bad);
    CKL();
    k_dg_target<D><<<ctx->nc, BLOCK, shm, ctx->stream>>>(ctx->geo, L, ctx->vg, d->gp, d->tp, d->W[c ^ 1], d->lam, 0,
                                                         d->bad);
    CKL();
    k_dg_update<D><<<ctx->nc, BLOCK, shm, ctx->stream>>>(ctx->geo, L, ctx->vg, d->gp, d->v[c], d->fv, d->v[c ^ 1], d->tp,
                                                         d->lam, d->q, 0);
    CKL();
    d->cur ^= 1;
  }
  return AVS_OK;
}

// Implicit steps: the interface stage of the explicit step (with r_f), the
// predictor's colour sweeps, the implicit flux, W^{n+1} and the target as in
// the explicit step, the micro right-hand side into the spare state buffer,
// the micro colour sweeps with the increment in the interface buffer (free
// once the right-hand side is formed), phi^{n+1} = phi^n + dphi.
template <int D>
avs_status dia_steps_implicit(avs_dia* d, int nsteps, int n_macro, int n_micro) {
  avs_ctx* ctx = d->ctx;
  const Leaves L = ctx->leaves(ctx->lcur);
  const unsigned gc = (unsigned)((ctx->nc + BLOCK - 1) / BLOCK), gf = (unsigned)((ctx->nf + BLOCK - 1) / BLOCK);
  const size_t shm = dia_shm(ctx);
  const int ncol = (int)ctx->col_off.size() - 1;
  for (int st = 0; st < nsteps; ++st) {
    const int c = d->cur;
    k_dg_recon<D><<<dim3((unsigned)round_up(ctx->nc, 8), (unsigned)((L.n + CHUNK - 1) / CHUNK)), BLOCK, 0,
                    ctx->stream>>>(ctx->geo, L, ctx->h, d->v[c], d->fv, d->gp, CHUNK);
    CKL();
    k_dg_face<D><<<ctx->nf, BLOCK, shm, ctx->stream>>>(ctx->geo, L, ctx->vg, ctx->gas, d->gp, ctx->h, d->fv, d->F,
                                                       d->bad, d->W[c], d->rf);
    CKL();
    k_imp_rhs<D, D + 3><<<gc, BLOCK, 0, ctx->stream>>>(ctx->geo, d->F, d->rf, d->irhs, d->idiag, d->dW);
    CKL();
    for (int sw = 0; sw < n_macro; ++sw)
      for (int t = 0; t < 2 * ncol; ++t) {
        const int cc = t < ncol ? t : 2 * ncol - 1 - t;
        const int cnt = ctx->col_off[cc + 1] - ctx->col_off[cc];
        k_dgi_macro<D><<<(unsigned)((cnt + BLOCK - 1) / BLOCK), BLOCK, 0, ctx->stream>>>(
            ctx->geo, ctx->gas, d->gp, ctx->dt, ctx->col_cells + ctx->col_off[cc], cnt, d->W[c], d->rf, d->irhs,
            d->idiag, d->dW, d->bad);
        CKL();
      }
    k_dgi_fhat<D><<<gf, BLOCK, 0, ctx->stream>>>(ctx->geo, d->gp, d->W[c], d->dW, d->rf, d->F);
    CKL();
    k_dg_macro<D><<<gc, BLOCK, 0, ctx->stream>>>(ctx->geo, ctx->gas, d->gp, ctx->dt, d->F, d->W[c], d->W[c ^ 1], d->q,
                                                 d->tp, d->bad);
    CKL();
    k_dg_target<D><<<ctx->nc, BLOCK, shm, ctx->stream>>>(ctx->geo, L, ctx->vg, d->gp, d->tp, d->W[c ^ 1], d->lam, 0,
                                                         d->bad);
    CKL();
    double* res = d->v[c ^ 1];
    double* dphi = d->fv;
    k_dg_update<D><<<ctx->nc, BLOCK, shm, ctx->stream>>>(ctx->geo, L, ctx->vg, d->gp, d->v[c], d->fv, res, d->tp,
                                                         d->lam, d->q, 2);
    CKL();
    k_imp_zero<double><<<ctx->nc, BLOCK, 0, ctx->stream>>>(3, ctx->nc, L, dphi);
    CKL();
    for (int sw = 0; sw < n_micro; ++sw)
      for (int t = 0; t < 2 * ncol; ++t) {
        const int cc = t < ncol ? t : 2 * ncol - 1 - t;
        const int cnt = ctx->col_off[cc + 1] - ctx->col_off[cc];
        // the backward half of the last sweep visits every cell for the last
        // time and writes phi^{n+1} over its right-hand side
        const bool last = sw == n_micro - 1 && t >= ncol;
        k_imp_micro<D, double, 3><<<(unsigned)cnt, BLOCK, 0, ctx->stream>>>(
            ctx->geo, L, ctx->col_cells + ctx->col_off[cc], res, dphi, d->tp, Dg<D>::NT, Dg<D>::IDT,
            last ? d->v[c] : nullptr, last ? d->v[c ^ 1] : nullptr);
        CKL();
      }
    if (n_micro == 0) {
      k_dgi_finish<<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->nc, L, d->v[c], dphi, d->v[c ^ 1]);
      CKL();
    }
    k_dg_heat<D><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->geo, L, d->v[c ^ 1], d->tp, d->q);
    CKL();
    d->cur ^= 1;
  }
  return AVS_OK;
}

template <int D>
avs_status dia_criterion(avs_dia* d, double C1, double C2, int nprobes) {
  avs_ctx* ctx = d->ctx;
  const Leaves L = ctx->leaves(ctx->lcur);
  const int nb = (L.n + BLOCK - 1) / BLOCK;
  k_dg_crit_partial<D><<<dim3(nb, ctx->ngrp), BLOCK, 0, ctx->stream>>>(L, ctx->nc, d->v[d->cur], d->W[d->cur],
                                                                      ctx->crit_part, nprobes, ctx->probe_cc,
                                                                      ctx->probe_prim, ctx->gas.R);
  CKL();
  k_crit_reduce<D><<<nb, BLOCK, 0, ctx->stream>>>(L, ctx->ngrp, ctx->crit_part, 0, ctx->probe_cc, ctx->probe_prim,
                                                 ctx->gas, C1, C2, ctx->lmax, ctx->Mk, ctx->raw);
  CKL();
  if (avs_status st = launch_sep_floor<D>(ctx, L)) return st;
  k_resolve<D><<<nb, BLOCK, 0, ctx->stream>>>(L, ctx->raw, ctx->eff, ctx->cnt);
  CKL();
  k_scan<<<1, BLOCK, 0, ctx->stream>>>(L.n, ctx->cnt, ctx->off);
  CKL();
  return AVS_OK;
}

template <int D>
avs_status dia_remap_state(avs_dia* d) {
  avs_ctx* ctx = d->ctx;
  const Leaves Lo = ctx->leaves(ctx->lcur), Ln = ctx->leaves(ctx->lcur ^ 1);
  const int c = d->cur;
  k_dg_gather<D><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->nc, Lo, Ln, ctx->pkind, ctx->psrc, d->v[c], d->v[c ^ 1]);
  CKL();
  k_dg_close<D><<<ctx->nc, BLOCK, dia_shm(ctx), ctx->stream>>>(ctx->geo, Ln, ctx->vg, d->gp, d->W[c], d->v[c ^ 1],
                                                               d->bad);
  CKL();
  // the heat fluxes of the remapped state for the next step's target
  const unsigned gc = (unsigned)((ctx->nc + BLOCK - 1) / BLOCK);
  k_dg_initrec<D><<<gc, BLOCK, 0, ctx->stream>>>(ctx->nc, d->gp, d->W[c], d->tp, d->bad);
  CKL();
  k_dg_heat<D><<<ctx->nc, BLOCK, 0, ctx->stream>>>(ctx->geo, Ln, d->v[c ^ 1], d->tp, d->q);
  CKL();
  return AVS_OK;
}
}  // namespace

extern "C" {

avs_status avs_dia_bytes(const avs_ctx* ctx, int64_t max_leaves, size_t* bytes) {
  if (!ctx || !bytes) return fail(AVS_E_INVALID, "null argument");
  if (max_leaves < ctx->nleaf[ctx->lcur] || max_leaves > ctx->cap)
    return fail(AVS_E_INVALID, "max_leaves must lie between the current leaf count and the leaf capacity");
  *bytes = dia_layout(ctx, max_leaves, nullptr, nullptr);
  return AVS_OK;
}

avs_status avs_dia_create(avs_ctx* ctx, const avs_rykov* gas, const double* prim0_host, int64_t max_leaves,
                          void* mem_dev, size_t mem_bytes, avs_dia** out) {
  if (!out) return fail(AVS_E_INVALID, "out is null");
  *out = nullptr;
  if (avs_status st = guard(ctx)) return st;
  if (ctx->prec != AVS_FP64) return fail(AVS_E_INVALID, "the diatomic path is FP64");
  if (!gas || !prim0_host || !mem_dev) return fail(AVS_E_INVALID, "null argument");
  if (((uintptr_t)mem_dev & 255)) return fail(AVS_E_INVALID, "mem_dev must be 256-byte aligned");
  if (!(gas->Z_rot >= 1.0 && std::isfinite(gas->Z_rot)) || !(gas->delta > 0.0 && gas->delta <= 1.0) ||
      !std::isfinite(gas->omega0) || !std::isfinite(gas->omega1))
    return fail(AVS_E_INVALID, "Rykov parameters: Z_rot >= 1, 0 < delta <= 1, finite omega_0 and omega_1");
  if (max_leaves < ctx->nleaf[ctx->lcur] || max_leaves > ctx->cap)
    return fail(AVS_E_INVALID, "max_leaves must lie between the current leaf count and the leaf capacity");
  if (dia_shm(ctx) > 48 * 1024) return fail(AVS_E_INVALID, "velocity grid too fine for the diatomic tables");
  const size_t need = dia_layout(ctx, max_leaves, nullptr, nullptr);
  if (mem_bytes < need) return fail(AVS_E_INVALID, "mem region too small (%zu < %zu)", mem_bytes, need);
  const int nc = ctx->nc, D = ctx->D, NW = D + 3;
  const double R = ctx->gas.R;
  std::vector<double> W0((size_t)nc * NW);
  for (int i = 0; i < nc; ++i) {
    const double* p = prim0_host + (size_t)i * NW;
    const double rho = p[0], Tt = p[1 + D], Tr = p[2 + D];
    double uu = 0.0;
    bool fin = std::isfinite(rho) && std::isfinite(Tt) && std::isfinite(Tr);
    for (int k = 0; k < D; ++k) {
      fin = fin && std::isfinite(p[1 + k]);
      uu += p[1 + k] * p[1 + k];
    }
    if (!(rho > 0 && Tt > 0 && Tr > 0) || !fin) return fail(AVS_E_INVALID, "cell %d: non-physical initial state", i);
    double* w = W0.data() + (size_t)i * NW;
    w[0] = rho;
    for (int k = 0; k < D; ++k) w[1 + k] = rho * p[1 + k];
    w[2 + D] = rho * R * Tr;
    w[1 + D] = 0.5 * rho * uu + 1.5 * rho * R * Tt + w[2 + D];
  }
  avs_dia* d = new avs_dia();
  d->ctx = ctx;
  d->gp = DiaGas{R, gas->Z_rot, gas->delta, gas->omega0, gas->omega1};
  dia_layout(ctx, max_leaves, d, (char*)mem_dev);
  d->gen = ctx->leaf_gen;
  d->max_leaves = max_leaves;
  const int badinit[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
  auto done = [&](avs_status st) { if (st) delete d; else *out = d; return st; };
  if (hipMemcpyAsync(d->W[0], W0.data(), sizeof(double) * W0.size(), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(d->bad, badinit, sizeof badinit, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
    return done(fail(AVS_E_HIP, "upload of the diatomic state failed"));
  avs_status st = D == 2 ? dia_init<2>(d) : dia_init<3>(d);
  if (!st) st = dia_check_bad(d);
  return done(st);
}

avs_status avs_dia_step(avs_dia* d, int32_t nsteps) {
  if (!d) return fail(AVS_E_INVALID, "null diatomic state");
  avs_ctx* ctx = d->ctx;
  if (avs_status st = guard(ctx)) return st;
  if (ctx->leaf_gen != d->gen) return fail(AVS_E_STATE, "the context's leaves changed since the diatomic state was made");
  if (nsteps < 0) return fail(AVS_E_INVALID, "nsteps < 0");
  if (avs_status st = ctx->D == 2 ? dia_steps<2>(d, nsteps) : dia_steps<3>(d, nsteps)) return st;
  return dia_check_bad(d);
}

avs_status avs_dia_step_implicit(avs_dia* d, int32_t nsteps, int32_t n_macro, int32_t n_micro) {
  if (!d) return fail(AVS_E_INVALID, "null diatomic state");
  avs_ctx* ctx = d->ctx;
  if (avs_status st = guard(ctx)) return st;
  if (ctx->leaf_gen != d->gen) return fail(AVS_E_STATE, "the context's leaves changed since the diatomic state was made");
  if (nsteps < 0 || n_macro < 0 || n_micro < 0) return fail(AVS_E_INVALID, "negative step or sweep count");
  // the micro increment lives in the interface buffer: [3][ncells][ld] must fit in [3][nfaces + 1][ld]
  if (ctx->nc > ctx->nf + 1) return fail(AVS_E_INVALID, "mesh has more cells than faces + 1");
  if (avs_status st = ctx->D == 2 ? dia_steps_implicit<2>(d, nsteps, n_macro, n_micro)
                                  : dia_steps_implicit<3>(d, nsteps, n_macro, n_micro))
    return st;
  return dia_check_bad(d);
}

avs_status avs_dia_get_state(avs_dia* d, double* vdf_host, double* W_host) {
  if (!d) return fail(AVS_E_INVALID, "null diatomic state");
  avs_ctx* ctx = d->ctx;
  if (avs_status st = guard(ctx)) return st;
  if (ctx->leaf_gen != d->gen) return fail(AVS_E_STATE, "the context's leaves changed since the diatomic state was made");
  const int n = ctx->nleaf[ctx->lcur], ld = ctx->ld[ctx->lcur], NW = ctx->D + 3;
  if (W_host)
    CK(hipMemcpyAsync(W_host, d->W[d->cur], sizeof(double) * ctx->nc * NW, hipMemcpyDeviceToHost, ctx->stream));
  if (vdf_host) {
    for (int p = 0; p < 3; ++p)
      CK(hipMemcpy2DAsync(vdf_host + (size_t)p * ctx->nc * n, n * sizeof(double),
                          d->v[d->cur] + (size_t)p * ctx->nc * ld, ld * sizeof(double), n * sizeof(double),
                          (size_t)ctx->nc, hipMemcpyDeviceToHost, ctx->stream));
  }
  CK(hipStreamSynchronize(ctx->stream));
  return AVS_OK;
}

avs_status avs_dia_adapt(avs_dia* d, double C1, double C2, const double* probes_host, int32_t nprobes,
                         int8_t* flags_dev, int64_t* n_new_host) {
  if (!d) return fail(AVS_E_INVALID, "null diatomic state");
  avs_ctx* ctx = d->ctx;
  if (avs_status st = guard(ctx)) return st;
  if (ctx->leaf_gen != d->gen) return fail(AVS_E_STATE, "the context's leaves changed since the diatomic state was made");
  if (std::isnan(C1) || std::isnan(C2)) return fail(AVS_E_INVALID, "C1/C2 must not be NaN");
  ctx->plan_valid = false;
  if (avs_status st = upload_probes(ctx, probes_host, nprobes, true)) return st;
  if (avs_status st = ctx->D == 2 ? dia_criterion<2>(d, C1, C2, nprobes) : dia_criterion<3>(d, C1, C2, nprobes))
    return st;
  int64_t nn = 0;
  if (avs_status st = finish_plan(ctx, flags_dev, &nn, nullptr)) return st;
  if (n_new_host) *n_new_host = nn;
  if (nn > d->max_leaves) {
    ctx->plan_valid = false;
    return fail(AVS_E_CAPACITY, "adaptation would produce %" PRId64 " leaves > the diatomic state's %" PRId64, nn,
                d->max_leaves);
  }
  ctx->plan_owner = d;
  return AVS_OK;
}

avs_status avs_dia_remap(avs_dia* d) {
  if (!d) return fail(AVS_E_INVALID, "null diatomic state");
  avs_ctx* ctx = d->ctx;
  if (avs_status st = guard(ctx)) return st;
  if (ctx->leaf_gen != d->gen) return fail(AVS_E_STATE, "the context's leaves changed since the diatomic state was made");
  if (!ctx->plan_valid) return fail(AVS_E_STATE, "no adaptation plan (call avs_dia_adapt first)");
  // a plan made by another adaptation (monatomic, batched, learned or another
  // diatomic state) was bounded by the context's capacity, not by these rows
  if (ctx->plan_owner != d)
    return fail(AVS_E_STATE, "the current plan was not made by avs_dia_adapt on this diatomic state");
  if (ctx->plan_n > d->max_leaves)
    return fail(AVS_E_CAPACITY, "plan of %d leaves > the diatomic state's %" PRId64, ctx->plan_n, d->max_leaves);
  if (avs_status st = ctx->D == 2 ? dia_remap_state<2>(d) : dia_remap_state<3>(d)) return st;
  // the context moves to the new leaves with its own (monatomic) state
  if (avs_status st = avs_remap(ctx, 0)) return st;
  const int c = d->cur;
  CK(hipMemcpyAsync(d->W[c ^ 1], d->W[c], sizeof(double) * ctx->nc * (ctx->D + 3), hipMemcpyDeviceToDevice,
                    ctx->stream));
  d->cur ^= 1;
  d->gen = ctx->leaf_gen;
  return dia_check_bad(d);
}

void avs_dia_destroy(avs_dia* d) { delete d; }

avs_status avs_moments(avs_ctx* ctx, double* fields_dev, double* totals_host) {
  if (avs_status st = guard(ctx)) return st;
  if (fields_dev) {
    if (avs_status st = DISPATCH(ctx, launch_moments, ctx)) return st;
    if (ctx->D == 2)
      k_fields<2><<<(ctx->nc + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->gas, ctx->W, ctx->q, fields_dev);
    else
      k_fields<3><<<(ctx->nc + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->gas, ctx->W, ctx->q, fields_dev);
    CKL();
  }
  if (totals_host) {
    if (ctx->D == 2)
      k_totals<2><<<1, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->geo.vol, ctx->W, ctx->tot);
    else
      k_totals<3><<<1, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->geo.vol, ctx->W, ctx->tot);
    CKL();
    CK(hipMemcpyAsync(totals_host, ctx->tot, sizeof(double) * (ctx->D + 2), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
  }
  return AVS_OK;
}

avs_status avs_moments_noalloc(avs_ctx* ctx, double* fields_dev, double* totals_host) {
  if (avs_status st = guard(ctx)) return st;
  if (totals_host) {
    const int nblk = (ctx->nc + NOALLOC_CELLS_PER_BLOCK - 1) / NOALLOC_CELLS_PER_BLOCK;
    if (nblk > NOALLOC_MAX_BLOCKS)
      return fail(AVS_E_CAPACITY, "avs_moments_noalloc: %d cells > its limit of %d", ctx->nc,
                  NOALLOC_MAX_BLOCKS * NOALLOC_CELLS_PER_BLOCK);
  }
  double* scr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES) scr = g_scratch_dev[ctx->device];
  }
  if (totals_host && !scr)
    return fail(AVS_E_HIP, "avs_moments_noalloc: the static scratch of device %d has no device address", ctx->device);
  if (fields_dev) {
    if (avs_status st = DISPATCH(ctx, launch_moments, ctx)) return st;
    if (ctx->D == 2)
      k_fields<2><<<(ctx->nc + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->gas, ctx->W, ctx->q, fields_dev);
    else
      k_fields<3><<<(ctx->nc + BLOCK - 1) / BLOCK, BLOCK, 0, ctx->stream>>>(ctx->nc, ctx->gas, ctx->W, ctx->q, fields_dev);
    CKL();
  }
  if (totals_host) {
    // partials of NOALLOC_CELLS_PER_BLOCK cells each, then their sum in block
    // order, staged at the end of the partials for the host copy; every
    // entry read is written first in the same call
    const int N = ctx->D + 2;
    const int nblk = (ctx->nc + NOALLOC_CELLS_PER_BLOCK - 1) / NOALLOC_CELLS_PER_BLOCK;
    double* part = scr;
    double* out = scr + (size_t)NOALLOC_MAX_BLOCKS * 5;
    if (ctx->D == 2) {
      k_totals_part<2><<<nblk, BLOCK, 0, ctx->stream>>>(ctx->nc, NOALLOC_CELLS_PER_BLOCK, ctx->geo.vol, ctx->W, part);
      CKL();
      k_totals<2><<<1, BLOCK, 0, ctx->stream>>>(nblk, nullptr, part, out);
    } else {
      k_totals_part<3><<<nblk, BLOCK, 0, ctx->stream>>>(ctx->nc, NOALLOC_CELLS_PER_BLOCK, ctx->geo.vol, ctx->W, part);
      CKL();
      k_totals<3><<<1, BLOCK, 0, ctx->stream>>>(nblk, nullptr, part, out);
    }
    CKL();
    CK(hipMemcpyAsync(totals_host, out, sizeof(double) * N, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
  }
  return AVS_OK;
}

static avs_status upload_probes(avs_ctx* ctx, const double* probes_host, int32_t nprobes, bool diatomic) {
  if (nprobes < 0 || nprobes > ctx->nprobe_max) return fail(AVS_E_INVALID, "nprobes must be in [0, %d]", ctx->nprobe_max);
  if (nprobes > 0 && !probes_host) return fail(AVS_E_INVALID, "probes_host is null");
  const int D = ctx->D, N = D + 2;
  std::vector<double> pcc((size_t)std::max(nprobes, 1) * N), Wp(N + 1);
  for (int p = 0; p < nprobes; ++p) {
    const double* pr = probes_host + (size_t)p * N;
    if (!(pr[0] > 0 && pr[1 + D] > 0)) return fail(AVS_E_INVALID, "probe %d is not a physical state", p);
    // the criterion's constants (rho, U, internal energy) come from the
    // probe's conserved state, as a cell's come from its W
    if (diatomic)
      conserved_dia_host(D, ctx->gas.R, pr, Wp.data());
    else
      conserved_host(D, ctx->gas.R, pr, Wp.data());
    crit_consts_host(D, Wp.data(), &pcc[(size_t)p * N]);
  }
  if (nprobes > 0) {
    CK(hipMemcpyAsync(ctx->probe_cc, pcc.data(), sizeof(double) * nprobes * N, hipMemcpyHostToDevice, ctx->stream));
    CK(hipMemcpyAsync(ctx->probe_prim, probes_host, sizeof(double) * nprobes * N, hipMemcpyHostToDevice, ctx->stream));
  }
  return AVS_OK;
}

// After the effective flags and their scan: new leaf count, capacity check,
// new leaf table and remap plan.  capacity_ok == nullptr: exceeding the
// capacity is an error; otherwise it is reported there and nothing is built.
static avs_status finish_plan(avs_ctx* ctx, int8_t* flags_dev, int64_t* n_new_host, bool* capacity_ok = nullptr) {
  int n_new = 0;
  const int n_old = ctx->nleaf[ctx->lcur];
  CK(hipMemcpyAsync(&n_new, ctx->off + n_old, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  if (flags_dev) CK(hipMemcpyAsync(flags_dev, ctx->eff, n_old, hipMemcpyDeviceToDevice, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  if (n_new_host) *n_new_host = n_new;
  if (n_new > ctx->cap) {
    if (capacity_ok) {
      *capacity_ok = false;
      return AVS_OK;
    }
    return fail(AVS_E_CAPACITY, "adaptation would produce %d leaves > leaf_capacity %" PRId64, n_new, ctx->cap);
  }
  if (capacity_ok) *capacity_ok = true;
  const int t = ctx->lcur ^ 1;
  ctx->nleaf[t] = n_new;
  ctx->ld[t] = (int)round_up(n_new, 64);
  if (avs_status st = DISPATCH_D(ctx, launch_scatter, ctx)) return st;
  CK(hipStreamSynchronize(ctx->stream));
  ctx->plan_n = n_new;
  ctx->plan_valid = true;
  ctx->plan_owner = nullptr;
  return AVS_OK;
}

avs_status avs_adapt(avs_ctx* ctx, double C1, double C2, const double* probes_host, int32_t nprobes, int8_t* flags_dev,
                     int64_t* n_new_host) {
  if (avs_status st = guard(ctx)) return st;
  if (std::isnan(C1) || std::isnan(C2)) return fail(AVS_E_INVALID, "C1/C2 must not be NaN");
  if (avs_status st = upload_probes(ctx, probes_host, nprobes)) return st;
  ctx->plan_valid = false;
  if (avs_status st = DISPATCH(ctx, launch_adapt, ctx, C1, C2, nprobes)) return st;
  return finish_plan(ctx, flags_dev, n_new_host);
}

avs_status avs_remap(avs_ctx* ctx, int32_t correction) {
  if (avs_status st = guard(ctx)) return st;
  if (!ctx->plan_valid) return fail(AVS_E_STATE, "no adaptation plan (call avs_adapt first)");
  if (correction < 0 || correction > 4) return fail(AVS_E_INVALID, "correction must be 0 to 4");
  if (avs_status st = DISPATCH(ctx, launch_remap, ctx, correction)) return st;
  ctx->lcur ^= 1;
  ctx->cur ^= 1;
  ++ctx->leaf_gen;
  ctx->plan_valid = false;
  if (avs_status st = DISPATCH_D(ctx, launch_bc_tables, ctx)) return st;
  if (!remap_leaves_moments(correction))
    if (avs_status st = DISPATCH(ctx, launch_moments, ctx)) return st;
  return check_bad(ctx);
}

avs_status avs_leaves(avs_ctx* ctx, int64_t* n_host, int64_t* ld_host, int32_t* level_host, int32_t* idx_host,
                      double* xi_host, double* w_host) {
  if (avs_status st = guard(ctx)) return st;
  const int t = ctx->lcur, n = ctx->nleaf[t], D = ctx->D;
  if (n_host) *n_host = n;
  if (ld_host) *ld_host = ctx->ld[t];
  std::vector<int> ib((size_t)D * n);
  std::vector<double> xb((size_t)D * n);
  if (level_host) CK(hipMemcpyAsync(level_host, ctx->lt[t].level, sizeof(int) * n, hipMemcpyDeviceToHost, ctx->stream));
  if (w_host) CK(hipMemcpyAsync(w_host, ctx->lt[t].w, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  for (int d = 0; d < D; ++d) {
    if (idx_host)
      CK(hipMemcpyAsync(ib.data() + (size_t)d * n, ctx->lt[t].idx + (size_t)d * ctx->cap, sizeof(int) * n,
                        hipMemcpyDeviceToHost, ctx->stream));
    if (xi_host)
      CK(hipMemcpyAsync(xb.data() + (size_t)d * n, ctx->lt[t].xi + (size_t)d * ctx->cap, sizeof(double) * n,
                        hipMemcpyDeviceToHost, ctx->stream));
  }
  CK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < n; ++k)
    for (int d = 0; d < D; ++d) {
      if (idx_host) idx_host[(size_t)k * D + d] = ib[(size_t)d * n + k];
      if (xi_host) xi_host[(size_t)k * D + d] = xb[(size_t)d * n + k];
    }
  return AVS_OK;
}

avs_status avs_plan(avs_ctx* ctx, int32_t* kind_host, int64_t* src_host, int32_t* child_host) {
  if (avs_status st = guard(ctx)) return st;
  if (!ctx->plan_valid) return fail(AVS_E_STATE, "no adaptation plan");
  const int n = ctx->plan_n;
  std::vector<int> s(n);
  if (kind_host) CK(hipMemcpyAsync(kind_host, ctx->pkind, sizeof(int) * n, hipMemcpyDeviceToHost, ctx->stream));
  if (child_host) CK(hipMemcpyAsync(child_host, ctx->pchild, sizeof(int) * n, hipMemcpyDeviceToHost, ctx->stream));
  if (src_host) CK(hipMemcpyAsync(s.data(), ctx->psrc, sizeof(int) * n, hipMemcpyDeviceToHost, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  if (src_host)
    for (int j = 0; j < n; ++j) src_host[j] = s[j];
  return AVS_OK;
}

avs_status avs_criterion(avs_ctx* ctx, double* Mk_host) {
  if (avs_status st = guard(ctx)) return st;
  if (!ctx->plan_valid) return fail(AVS_E_STATE, "no adaptation result");
  if (!Mk_host) return fail(AVS_E_INVALID, "Mk_host is null");
  CK(hipMemcpyAsync(Mk_host, ctx->Mk, sizeof(double) * ctx->nleaf[ctx->lcur], hipMemcpyDeviceToHost, ctx->stream));
  CK(hipStreamSynchronize(ctx->stream));
  return AVS_OK;
}

avs_status avs_set_leaves(avs_ctx* ctx, int64_t n, const int32_t* level_host, const int32_t* idx_host) {
  if (avs_status st = guard(ctx)) return st;
  if (n < 1 || n > ctx->cap) return fail(AVS_E_INVALID, "leaf count %" PRId64 " outside [1, capacity]", n);
  if (!level_host || !idx_host) return fail(AVS_E_INVALID, "null leaf arrays");
  const int D = ctx->D;
  // a valid leaf set tiles the forest: in-range cells, increasing disjoint Morton ranges, full cover
  uint64_t next = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int l = level_host[k];
    if (l < 0 || l > ctx->lmax) return fail(AVS_E_INVALID, "leaf %" PRId64 ": level out of range", k);
    for (int d = 0; d < D; ++d)
      if (idx_host[k * D + d] < 0 || idx_host[k * D + d] >= (ctx->base[d] << l))
        return fail(AVS_E_INVALID, "leaf %" PRId64 ": index out of range", k);
    const uint64_t key = morton(D, ctx->lmax, l, idx_host + k * D);
    if (k > 0 && key < next) return fail(AVS_E_INVALID, "leaf %" PRId64 " overlaps or is out of depth-first order", k);
    next = key + (1ull << (D * (ctx->lmax - l)));
  }
  uint64_t total = 1;
  for (int d = 0; d < D; ++d) total *= (uint64_t)ctx->base[d] << ctx->lmax;
  // disjoint in-box cells whose volumes add up to the box tile it
  uint64_t covered = 0;
  for (int64_t k = 0; k < n; ++k) covered += 1ull << (D * (ctx->lmax - level_host[k]));
  if (covered != total) return fail(AVS_E_INVALID, "leaves do not cover the velocity box");
  std::vector<int> lev(level_host, level_host + n);
  const int t = ctx->lcur ^ 1;
  if (avs_status st = upload_leaves(ctx, t, (int)n, lev.data(), idx_host)) return st;
  ctx->lcur = t;
  ctx->plan_valid = false;
  if (avs_status st = DISPATCH(ctx, launch_init_vdf, ctx)) return st;
  if (avs_status st = DISPATCH_D(ctx, launch_bc_tables, ctx)) return st;
  if (avs_status st = DISPATCH(ctx, launch_moments, ctx)) return st;
  return check_bad(ctx);
}

avs_status avs_get_state(avs_ctx* ctx, double* vdf_host, double* W_host) {
  if (avs_status st = guard(ctx)) return st;
  const int n = ctx->nleaf[ctx->lcur], ld = ctx->ld[ctx->lcur], N = ctx->D + 2;
  if (W_host) CK(hipMemcpyAsync(W_host, ctx->W, sizeof(double) * ctx->nc * N, hipMemcpyDeviceToHost, ctx->stream));
  if (vdf_host) {
    const size_t es = ctx->esize(), cs = (size_t)ctx->nc * ld;
    if (ctx->prec == AVS_FP64) {
      CK(hipMemcpy2DAsync(vdf_host, n * es, ctx->vdf[ctx->cur], ld * es, n * es, (size_t)ctx->P * ctx->nc,
                          hipMemcpyDeviceToHost, ctx->stream));
    } else {
      std::vector<float> tmp((size_t)ctx->P * ctx->nc * n);
      CK(hipMemcpy2DAsync(tmp.data(), n * es, ctx->vdf[ctx->cur], ld * es, n * es, (size_t)ctx->P * ctx->nc,
                          hipMemcpyDeviceToHost, ctx->stream));
      CK(hipStreamSynchronize(ctx->stream));
      for (size_t t = 0; t < tmp.size(); ++t) vdf_host[t] = tmp[t];
    }
    (void)cs;
  }
  CK(hipStreamSynchronize(ctx->stream));
  return AVS_OK;
}

avs_status avs_set_state(avs_ctx* ctx, const double* vdf_host, const double* W_host) {
  if (avs_status st = guard(ctx)) return st;
  if (!W_host && !vdf_host) return fail(AVS_E_INVALID, "W_host or vdf_host is required");
  const int n = ctx->nleaf[ctx->lcur], ld = ctx->ld[ctx->lcur], D = ctx->D, N = D + 2;
  auto physical = [&](const double* W) {
    for (int i = 0; i < ctx->nc; ++i) {
      const double* w = W + (size_t)i * N;
      double ke = 0;
      for (int d = 0; d < D; ++d) ke += w[1 + d] * w[1 + d];
      if (!(w[0] > 0) || !(w[1 + D] - 0.5 * ke / w[0] > 0)) return i;
    }
    return -1;
  };
  if (W_host) {
    const int bad_cell = physical(W_host);
    if (bad_cell >= 0) return fail(AVS_E_INVALID, "W of cell %d is not physical", bad_cell);
    CK(hipMemcpyAsync(ctx->W, W_host, sizeof(double) * ctx->nc * N, hipMemcpyHostToDevice, ctx->stream));
  }
  if (vdf_host) {
    const size_t es = ctx->esize();
    if (ctx->prec == AVS_FP64) {
      CK(hipMemcpy2DAsync(ctx->vdf[ctx->cur], ld * es, vdf_host, n * es, n * es, (size_t)ctx->P * ctx->nc,
                          hipMemcpyHostToDevice, ctx->stream));
      CK(hipStreamSynchronize(ctx->stream));
    } else {
      std::vector<float> tmp;
      copy_from_host(tmp, vdf_host, (size_t)ctx->P * ctx->nc * n);
      CK(hipMemcpy2DAsync(ctx->vdf[ctx->cur], ld * es, tmp.data(), n * es, n * es, (size_t)ctx->P * ctx->nc,
                          hipMemcpyHostToDevice, ctx->stream));
      CK(hipStreamSynchronize(ctx->stream));
    }
  } else {
    if (avs_status st = DISPATCH(ctx, launch_init_vdf, ctx)) return st;
  }
  ctx->plan_valid = false;
  if (avs_status st = DISPATCH(ctx, launch_moments, ctx)) return st;
  if (!W_host) {
    // W from the moments of the given VDF
    std::vector<double> Wm((size_t)ctx->nc * N);
    CK(hipMemcpyAsync(Wm.data(), ctx->mom, sizeof(double) * Wm.size(), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    const int bad_cell = physical(Wm.data());
    if (bad_cell >= 0) {
      ctx->failed = true;
      return fail(AVS_E_NUMERIC, "moments of the given VDF are not physical in cell %d", bad_cell);
    }
    CK(hipMemcpyAsync(ctx->W, Wm.data(), sizeof(double) * Wm.size(), hipMemcpyHostToDevice, ctx->stream));
    if (avs_status st = DISPATCH(ctx, launch_moments, ctx)) return st;   // q and the target's moments about the new W
  }
  return check_bad(ctx);
}

avs_status avs_get_cells(avs_ctx* ctx, int64_t ncell_sel, const int64_t* cells_host, double* vdf_host) {
  if (avs_status st = guard(ctx)) return st;
  if (ncell_sel < 0 || (ncell_sel > 0 && (!cells_host || !vdf_host))) return fail(AVS_E_INVALID, "bad selection");
  const int n = ctx->nleaf[ctx->lcur], ld = ctx->ld[ctx->lcur];
  const size_t es = ctx->esize(), cs = (size_t)ctx->nc * ld;
  std::vector<char> tmp((size_t)n * es);
  for (int64_t r = 0; r < ncell_sel; ++r) {
    const int64_t c = cells_host[r];
    if (c < 0 || c >= ctx->nc) return fail(AVS_E_INVALID, "cell %" PRId64 " out of range", c);
    for (int p = 0; p < ctx->P; ++p) {
      const char* src = (const char*)ctx->vdf[ctx->cur] + ((size_t)p * cs + (size_t)c * ld) * es;
      CK(hipMemcpyAsync(tmp.data(), src, n * es, hipMemcpyDeviceToHost, ctx->stream));
      CK(hipStreamSynchronize(ctx->stream));
      double* o = vdf_host + ((size_t)p * ncell_sel + r) * n;
      if (ctx->prec == AVS_FP64)
        memcpy(o, tmp.data(), n * es);
      else
        for (int k = 0; k < n; ++k) o[k] = ((const float*)tmp.data())[k];
    }
  }
  return AVS_OK;
}

avs_status avs_profile(avs_ctx* ctx, int32_t enable) {
  if (avs_status st = guard(ctx)) return st;
  CK(hipStreamSynchronize(ctx->stream));
  if (enable) {
    ctx->evused = 0;
    ctx->evrec.clear();
  }
  ctx->prof = enable != 0;
  return AVS_OK;
}

int32_t avs_profile_read(avs_ctx* ctx, int32_t nmax, char* names_host, double* ms_host, int64_t* count_host) {
  if (guard(ctx)) return -1;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return -1;
  double ms[K_NKERNELS] = {0};
  int64_t cnt[K_NKERNELS] = {0};
  for (const auto& r : ctx->evrec) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ctx->evpool[r.second], ctx->evpool[r.second + 1]) == hipSuccess) {
      ms[r.first] += t;
      cnt[r.first] += 1;
    }
  }
  int n = 0;
  for (int k = 0; k < K_NKERNELS && n < nmax; ++k) {
    if (!cnt[k]) continue;
    if (names_host) snprintf(names_host + 32 * n, 32, "%s", kKernelNames[k]);
    if (ms_host) ms_host[n] = ms[k];
    if (count_host) count_host[n] = cnt[k];
    ++n;
  }
  return n;
}


size_t avs_batch_workspace_bytes(int32_t ncase) {
  if (ncase < 1 || ncase > 4096) return 0;
  return batch_args_bytes(ncase) + batch_offs_bytes(ncase) + remap_args_bytes(ncase) + remap_offs_bytes(ncase);
}

avs_status avs_batch_create(int32_t ncase, avs_ctx* const* ctxs, void* workspace_dev, size_t workspace_bytes,
                            avs_batch** out) {
  if (!out) return fail(AVS_E_INVALID, "out is null");
  *out = nullptr;
  if (ncase < 1 || ncase > 4096 || !ctxs) return fail(AVS_E_INVALID, "ncase must be in [1, 4096]");
  if (!workspace_dev || workspace_bytes < avs_batch_workspace_bytes(ncase))
    return fail(AVS_E_INVALID, "batch workspace too small (%zu < %zu)", workspace_bytes, avs_batch_workspace_bytes(ncase));
  for (int i = 0; i < ncase; ++i) {
    avs_ctx* c = ctxs[i];
    if (avs_status st = guard(c)) return st;
    if (c->D != ctxs[0]->D || c->prec != ctxs[0]->prec)
      return fail(AVS_E_INVALID, "case %d: all cases of a batch need the same dimension and precision", i);
    if (c->stream != ctxs[0]->stream) return fail(AVS_E_INVALID, "case %d: all cases of a batch need the same stream", i);
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(AVS_E_INVALID, "case %d appears twice", i);
  }
  if (ctxs[0]->stream == nullptr) return fail(AVS_E_INVALID, "a batch needs a non-default stream (graph capture)");
  avs_batch* b = new avs_batch();
  b->cases.assign(ctxs, ctxs + ncase);
  b->D = ctxs[0]->D;
  b->prec = ctxs[0]->prec;
  b->stream = ctxs[0]->stream;
  b->ws = (char*)workspace_dev;
  *out = b;
  return AVS_OK;
}

avs_status avs_batch_step(avs_batch* b, int32_t nsteps, int32_t use_graph) {
  if (!b) return fail(AVS_E_INVALID, "null batch");
  if (nsteps < 0) return fail(AVS_E_INVALID, "nsteps < 0");
  for (avs_ctx* c : b->cases)
    if (avs_status st = guard(c)) return st;
  if (nsteps == 0) return AVS_OK;
  avs_status st = batch_run(b, nsteps, use_graph != 0);
  if (st)
    for (avs_ctx* c : b->cases) c->failed = true;
  return st;
}

namespace {

constexpr int kSideStreams = 4;

// Make the side streams wait for the work enqueued so far on the batch's
// stream (created on first use).
avs_status side_fork(avs_batch* b) {
  avs_ctx* ctx = nullptr;
  if (b->side.empty()) {
    for (int j = 0; j < kSideStreams; ++j) {
      hipStream_t q = nullptr;
      CK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
      b->side.push_back(q);
    }
    for (int j = 0; j <= kSideStreams; ++j) {
      hipEvent_t e = nullptr;
      CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->side_ev.push_back(e);
    }
  }
  CK(hipEventRecord(b->side_ev[kSideStreams], b->stream));
  for (hipStream_t q : b->side) CK(hipStreamWaitEvent(q, b->side_ev[kSideStreams], 0));
  return AVS_OK;
}

// Make the batch's stream wait for everything enqueued on the side streams.
avs_status side_join(avs_batch* b) {
  avs_ctx* ctx = nullptr;
  for (int j = 0; j < (int)b->side.size(); ++j) {
    CK(hipEventRecord(b->side_ev[j], b->side[j]));
    CK(hipStreamWaitEvent(b->stream, b->side_ev[j], 0));
  }
  return AVS_OK;
}

// Joins the side streams back on every way out of a call that forked them,
// so that the batch's stream never runs ahead of side-stream work.
struct SideJoin {
  avs_batch* b;
  ~SideJoin() { (void)side_join(b); }
};

// A case's launches go to side stream i % kSideStreams while this lives.
struct OnSide {
  avs_ctx* c;
  hipStream_t keep;
  OnSide(avs_batch* b, int i) : c(b->cases[i]), keep(c->stream) { c->stream = b->side[i % b->side.size()]; }
  ~OnSide() { c->stream = keep; }
};

}  // namespace

avs_status avs_batch_adapt(avs_batch* b, const double* C1_host, const double* C2_host, int64_t* n_new_host) {
  avs_ctx* ctx = nullptr;
  if (!b) return fail(AVS_E_INVALID, "null batch");
  if (!C1_host || !C2_host) return fail(AVS_E_INVALID, "null C1/C2 arrays");
  const int n = (int)b->cases.size();
  for (int i = 0; i < n; ++i) {
    if (avs_status st = guard(b->cases[i])) return st;
    if (std::isnan(C1_host[i]) || std::isnan(C2_host[i])) return fail(AVS_E_INVALID, "case %d: C1/C2 must not be NaN", i);
  }
  // criterion, flags, scan of every case, side by side; one wait for the counts
  for (avs_ctx* c : b->cases) c->plan_valid = false;
  if (avs_status st = side_fork(b)) return st;
  {
    SideJoin join{b};
    for (int i = 0; i < n; ++i) {
      OnSide on(b, i);
      avs_ctx* c = b->cases[i];
      if (avs_status st = DISPATCH(c, launch_adapt, c, C1_host[i], C2_host[i], 0)) return st;
    }
  }
  std::vector<int> nn(n, 0);
  for (int i = 0; i < n; ++i) {
    avs_ctx* c = b->cases[i];
    CK(hipMemcpyAsync(&nn[i], c->off + c->nleaf[c->lcur], sizeof(int), hipMemcpyDeviceToHost, b->stream));
  }
  CK(hipStreamSynchronize(b->stream));
  for (int i = 0; i < n; ++i) {
    if (n_new_host) n_new_host[i] = nn[i];
    if (nn[i] > b->cases[i]->cap)
      return fail(AVS_E_CAPACITY, "case %d: adaptation would produce %d leaves > leaf_capacity %" PRId64, i, nn[i],
                  b->cases[i]->cap);
  }
  if (avs_status st = side_fork(b)) return st;
  {
    SideJoin join{b};
    for (int i = 0; i < n; ++i) {
      OnSide on(b, i);
      avs_ctx* c = b->cases[i];
      const int t = c->lcur ^ 1;
      c->nleaf[t] = nn[i];
      c->ld[t] = (int)round_up(nn[i], 64);
      if (avs_status st = DISPATCH_D(c, launch_scatter, c)) return st;
    }
  }
  CK(hipStreamSynchronize(b->stream));
  for (int i = 0; i < n; ++i) {
    b->cases[i]->plan_n = nn[i];
    b->cases[i]->plan_valid = true;
    b->cases[i]->plan_owner = nullptr;
  }
  return AVS_OK;
}

extern "C++" {
namespace {

// The remap of every member in five launches over all members' workgroups:
// gather (+ W'), correction (correction 1, 2), the boundary pair and face
// tables of the new leaves, the moments of the new state.  The members'
// leaf and state buffers flip as after avs_remap.
template <int D, typename T>
avs_status batch_remap_launch(avs_batch* b, int correction) {
  avs_ctx* ctx = nullptr;
  const int n = (int)b->cases.size();
  char* base = b->ws + batch_args_bytes(n) + batch_offs_bytes(n);
  b->host_remap.resize(remap_args_bytes(n) + remap_offs_bytes(n));
  RemapArgs<T>* args = reinterpret_cast<RemapArgs<T>*>(b->host_remap.data());
  int* off = reinterpret_cast<int*>(b->host_remap.data() + remap_args_bytes(n));
  for (int k = 0; k < BR_N; ++k) off[k * (n + 1)] = 0;
  int numax = 0;
  for (int i = 0; i < n; ++i) {
    avs_ctx* c = b->cases[i];
    RemapArgs<T> a;
    a.g = c->geo;
    a.Lo = c->leaves(c->lcur);
    a.Ln = c->leaves(c->lcur ^ 1);
    a.vg = c->vg;
    a.gas = c->gas;
    a.pkind = c->pkind;
    a.psrc = c->psrc;
    a.vin = (const T*)c->vdf[c->cur];
    a.vout = (T*)c->vdf[c->cur ^ 1];
    a.momp = c->momp;
    a.W = c->W;
    a.mom = c->mom;
    a.q = c->q;
    a.bad = c->bad;
    a.bcpair = c->bcpair;
    a.bden = c->bden;
    a.bfin = c->bfin;
    a.nbl = (a.Ln.n + BLOCK - 1) / BLOCK;
    args[i] = a;
    numax = std::max(numax, c->vg.numax);
    // the correction kernel forms the moments of the new state itself
    const int cnt[BR_N] = {c->nc, correction > 0 ? c->nc : 0, c->nbc > 0 ? a.nbl * c->nbc : 0, c->n_bnd,
                           remap_leaves_moments(correction) ? 0 : c->nc};
    for (int k = 0; k < BR_N; ++k) off[k * (n + 1) + i + 1] = off[k * (n + 1) + i] + cnt[k];
  }
  CK(hipMemcpyAsync(base, b->host_remap.data(), b->host_remap.size(), hipMemcpyHostToDevice, b->stream));
  const RemapArgs<T>* a = reinterpret_cast<const RemapArgs<T>*>(base);
  const int* o = reinterpret_cast<const int*>(base + remap_args_bytes(n));
  auto nb = [&](int k) { return off[k * (n + 1) + n]; };
  if (nb(BR_GATHER) > 0) {
    kb_remap_gather<D, T><<<nb(BR_GATHER), BLOCK, 0, b->stream>>>(a, o + BR_GATHER * (n + 1), n);
    CKL();
  }
  if (nb(BR_CORRECT) > 0) {
    kb_remap_correct<D, T><<<nb(BR_CORRECT), BLOCK, (size_t)2 * D * numax * sizeof(double), b->stream>>>(
        a, o + BR_CORRECT * (n + 1), n, correction);
    CKL();
  }
  if (nb(BR_PAIRS) > 0) {
    kb_bc_pairs<D, T><<<nb(BR_PAIRS), BLOCK, 0, b->stream>>>(a, o + BR_PAIRS * (n + 1), n);
    CKL();
  }
  if (nb(BR_BND) > 0) {
    kb_bnd_tables<D, T><<<nb(BR_BND), BLOCK, 0, b->stream>>>(a, o + BR_BND * (n + 1), n);
    CKL();
  }
  if (nb(BR_MOM) > 0) {
    kb_cell_moments<D, T><<<nb(BR_MOM), BLOCK, 0, b->stream>>>(a, o + BR_MOM * (n + 1), n);
    CKL();
  }
  for (avs_ctx* c : b->cases) {
    c->lcur ^= 1;
    c->cur ^= 1;
    ++c->leaf_gen;
    c->plan_valid = false;
  }
  // the host records stay in use until the copy has read them
  CK(hipStreamSynchronize(b->stream));
  return AVS_OK;
}

}  // namespace
}  // extern "C++"

avs_status avs_batch_remap(avs_batch* b, int32_t correction) {
  if (!b) return fail(AVS_E_INVALID, "null batch");
  if (correction < 0 || correction > 4) return fail(AVS_E_INVALID, "correction must be 0 to 4");
  const int n = (int)b->cases.size();
  for (int i = 0; i < n; ++i) {
    if (avs_status st = guard(b->cases[i])) return st;
    if (!b->cases[i]->plan_valid) return fail(AVS_E_STATE, "case %d: no adaptation plan", i);
  }
  avs_ctx* ctx = nullptr;
  if (correction <= 2) {
    // one set of launches over all members
    if (avs_status st = b->D == 2 ? (b->prec == AVS_FP64 ? batch_remap_launch<2, double>(b, correction)
                                                          : batch_remap_launch<2, float>(b, correction))
                                  : (b->prec == AVS_FP64 ? batch_remap_launch<3, double>(b, correction)
                                                          : batch_remap_launch<3, float>(b, correction)))
      return st;
    for (avs_ctx* c : b->cases)
      if (avs_status st = check_bad(c)) return st;
    return AVS_OK;
  }
  // the equilibrium bypass: each member's own kernels, side by side
  if (avs_status st = side_fork(b)) return st;
  {
    SideJoin join{b};
    for (int i = 0; i < n; ++i) {
      OnSide on(b, i);
      avs_ctx* c = b->cases[i];
      if (avs_status st = DISPATCH(c, launch_remap, c, correction)) return st;
      c->lcur ^= 1;
      c->cur ^= 1;
      ++c->leaf_gen;
      c->plan_valid = false;
      if (avs_status st = DISPATCH_D(c, launch_bc_tables, c)) return st;
      if (!remap_leaves_moments(correction))
        if (avs_status st = DISPATCH(c, launch_moments, c)) return st;
    }
  }
  CK(hipStreamSynchronize(b->stream));
  for (avs_ctx* c : b->cases)
    if (avs_status st = check_bad(c)) return st;
  return AVS_OK;
}

avs_status avs_batch_check(avs_batch* b) {
  if (!b) return fail(AVS_E_INVALID, "null batch");
  for (avs_ctx* c : b->cases)
    if (avs_status st = check_bad(c)) return st;
  return AVS_OK;
}

avs_status avs_batch_tune(avs_batch* b, int32_t* chunk_host) {
  if (!b) return fail(AVS_E_INVALID, "null batch");
  avs_ctx* ctx = nullptr;
  const int cand[] = {512, 1024, 2048, 4096, 8192, 16384};
  bool present[4] = {false, false, false, false};
  for (avs_ctx* c : b->cases) present[leaf_bucket(c->nleaf[c->lcur])] = true;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  // time of two dry steps (the cases' state is left as it was)
  auto timed = [&](float& ms) -> avs_status {
    if (avs_status st = batch_dry_step(b)) return st;     // warm the choice
    CK(hipEventRecord(e0, b->stream));
    for (int r = 0; r < 2; ++r)
      if (avs_status st = batch_dry_step(b)) return st;
    CK(hipEventRecord(e1, b->stream));
    CK(hipEventSynchronize(e1));
    CK(hipEventElapsedTime(&ms, e0, e1));
    return AVS_OK;
  };
  // knob 1: pass-A leaf chunk, one bucket at a time, the others at their
  // current choice
  for (int q = 0; q < 4; ++q) {
    if (!present[q]) continue;
    float best = 1e30f;
    int arg = b->chunk[q];
    for (int c : cand) {
      b->chunk[q] = c;
      float ms = 0.f;
      if (avs_status st = timed(ms)) return st;
      if (ms < best) {
        best = ms;
        arg = c;
      }
    }
    b->chunk[q] = arg;
  }
  // knob 2: pass C with one or two leaves' loads in flight
  {
    float best = 1e30f;
    int arg = b->passc_two;
    for (int v : {0, 1}) {
      b->passc_two = v;
      float ms = 0.f;
      if (avs_status st = timed(ms)) return st;
      if (ms < best) {
        best = ms;
        arg = v;
      }
    }
    b->passc_two = arg;
  }
  CK(hipStreamSynchronize(b->stream));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (chunk_host) {
    for (int q = 0; q < 4; ++q) chunk_host[q] = b->chunk[q];
    chunk_host[4] = b->passc_two;
  }
  return AVS_OK;
}

void avs_batch_destroy(avs_batch* b) { delete b; }

// ------------------------------------------------------------ learned proposal
struct avs_mlp {
  float *prm, *m, *v, *grad;
  uint16_t* wbf;
  float* gpart;
  double *lossp, *loss;
  int64_t max_batch;
  int maxtile;
  double rho_ref, T_ref;
  hipStream_t stream;
  int64_t t = 0;
  bool failed = false;
};

static void mlp_carve(avs_mlp& x, Carver& c) {
  using namespace mlp;
  x.prm = c.take<float>(NPARAM);
  x.m = c.take<float>(NPARAM);
  x.v = c.take<float>(NPARAM);
  x.grad = c.take<float>(NPARAM);
  x.wbf = c.take<uint16_t>(PWN);
  x.gpart = c.take<float>((size_t)x.maxtile * GN);
  x.lossp = c.take<double>(x.maxtile);
  x.loss = c.take<double>(1);
}

#define MCK(expr)                                                                                  \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      mlp->failed = true;                                                                          \
      return fail(AVS_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    }                                                                                              \
  } while (0)

static avs_status mlp_guard(const avs_mlp* mlp) {
  if (!mlp) return fail(AVS_E_INVALID, "null network");
  if (mlp->failed) return fail(AVS_E_STATE, "network is in the failed state after an earlier device error");
  return AVS_OK;
}

// Dynamic LDS above the default limit for the fused tile kernel.
static hipError_t mlp_lds_attr() {
  using namespace mlp;
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_mlp_tile<FWD_LOGITS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)LDS_BYTES);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_mlp_tile<FWD_FLAGS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_BYTES);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_mlp_tile<TRAIN>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_BYTES);
  done = e == hipSuccess;
  return e;
}

static avs_status mlp_upload(avs_mlp* mlp, const float* params_host) {
  using namespace mlp;
  MCK(hipMemcpyAsync(mlp->prm, params_host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, mlp->stream));
  MCK(hipMemsetAsync(mlp->m, 0, sizeof(float) * NPARAM, mlp->stream));
  MCK(hipMemsetAsync(mlp->v, 0, sizeof(float) * NPARAM, mlp->stream));
  k_mlp_pack<<<(PWN + TPB - 1) / TPB, TPB, 0, mlp->stream>>>(mlp->prm, mlp->wbf);
  MCK(hipGetLastError());
  MCK(hipStreamSynchronize(mlp->stream));
  mlp->t = 0;
  return AVS_OK;
}

static avs_status mlp_grad_into(avs_mlp* mlp, const uint16_t* feat, const int8_t* flags, const int32_t* rows, int64_t n,
                                float* grad) {
  using namespace mlp;
  const int nt = (int)((n + TILE - 1) / TILE);
  MCK(mlp_lds_attr());
  k_mlp_tile<TRAIN><<<nt, TPB, LDS_BYTES, mlp->stream>>>((int)n, feat, rows, mlp->wbf, mlp->prm, nullptr, nullptr, 0,
                                                         nullptr, flags, (float)(1.0 / (double)n), mlp->gpart,
                                                         mlp->lossp);
  MCK(hipGetLastError());
  k_mlp_reduce<<<(NPARAM + TPB - 1) / TPB, TPB, 0, mlp->stream>>>(nt, mlp->gpart, mlp->lossp, 1.0 / (double)n, grad,
                                                                  mlp->loss);
  MCK(hipGetLastError());
  return AVS_OK;
}

static avs_status mlp_check_batch(const avs_mlp* mlp, const uint16_t* feat, const int8_t* flags, int64_t n) {
  if (!feat || !flags) return fail(AVS_E_INVALID, "null features or labels");
  if (n < 1 || n > mlp->max_batch) return fail(AVS_E_INVALID, "batch of %" PRId64 " rows outside [1, %" PRId64 "]", n, mlp->max_batch);
  return AVS_OK;
}

static avs_status mlp_check_adam(const avs_adam* hp) {
  if (!hp) return fail(AVS_E_INVALID, "null Adam parameters");
  if (!(hp->lr > 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) || !(hp->beta2 >= 0 && hp->beta2 < 1) || !(hp->eps > 0))
    return fail(AVS_E_INVALID, "Adam parameters need lr > 0, 0 <= beta < 1, eps > 0");
  return AVS_OK;
}

static avs_status mlp_adam_launch(avs_mlp* mlp, const float* grad, const avs_adam* hp) {
  using namespace mlp;
  const int64_t t = mlp->t + 1;
  const double c1 = 1.0 / (1.0 - std::pow(hp->beta1, (double)t)), c2 = 1.0 / (1.0 - std::pow(hp->beta2, (double)t));
  k_mlp_adam<<<(NPARAM + TPB - 1) / TPB, TPB, 0, mlp->stream>>>(grad, mlp->prm, mlp->m, mlp->v, hp->lr, hp->beta1,
                                                                hp->beta2, hp->eps, c1, c2, mlp->wbf);
  MCK(hipGetLastError());
  k_mlp_pack<<<(PWN + TPB - 1) / TPB, TPB, 0, mlp->stream>>>(mlp->prm, mlp->wbf);
  MCK(hipGetLastError());
  mlp->t = t;
  return AVS_OK;
}

int64_t avs_mlp_param_count(void) { return mlp::NPARAM; }

size_t avs_mlp_state_bytes(int64_t max_batch) {
  if (max_batch < 1 || max_batch > ((int64_t)1 << 26)) {
    fail(AVS_E_INVALID, "max_batch must be in [1, 2^26]");
    return 0;
  }
  avs_mlp x{};
  x.maxtile = (int)((max_batch + mlp::TILE - 1) / mlp::TILE);
  Carver c{nullptr};
  mlp_carve(x, c);
  return c.off;
}

avs_status avs_mlp_create(const float* params_host, int64_t max_batch, double rho_ref, double T_ref, void* state_dev,
                          size_t state_bytes, void* hip_stream, avs_mlp** out) {
  if (!out) return fail(AVS_E_INVALID, "out is null");
  *out = nullptr;
  if (!params_host || !state_dev) return fail(AVS_E_INVALID, "null parameters or state");
  const size_t need = avs_mlp_state_bytes(max_batch);
  if (need == 0) return AVS_E_INVALID;
  if (state_bytes < need) return fail(AVS_E_INVALID, "network state too small (%zu < %zu)", state_bytes, need);
  if ((uintptr_t)state_dev % 256) return fail(AVS_E_INVALID, "network state must be 256-byte aligned");
  if (!(rho_ref > 0) || !(T_ref > 0)) return fail(AVS_E_INVALID, "rho_ref and T_ref must be positive");
  avs_mlp* mlp = new avs_mlp();
  mlp->max_batch = max_batch;
  mlp->maxtile = (int)((max_batch + mlp::TILE - 1) / mlp::TILE);
  mlp->rho_ref = rho_ref;
  mlp->T_ref = T_ref;
  mlp->stream = (hipStream_t)hip_stream;
  Carver c{(char*)state_dev};
  mlp_carve(*mlp, c);
  if (avs_status st = mlp_upload(mlp, params_host)) {
    delete mlp;
    return st;
  }
  *out = mlp;
  return AVS_OK;
}

avs_status avs_mlp_get_params(avs_mlp* mlp, float* params_host) {
  if (avs_status st = mlp_guard(mlp)) return st;
  if (!params_host) return fail(AVS_E_INVALID, "params_host is null");
  MCK(hipMemcpyAsync(params_host, mlp->prm, sizeof(float) * mlp::NPARAM, hipMemcpyDeviceToHost, mlp->stream));
  MCK(hipStreamSynchronize(mlp->stream));
  return AVS_OK;
}

avs_status avs_mlp_set_params(avs_mlp* mlp, const float* params_host) {
  if (avs_status st = mlp_guard(mlp)) return st;
  if (!params_host) return fail(AVS_E_INVALID, "params_host is null");
  return mlp_upload(mlp, params_host);
}

avs_status avs_mlp_forward(avs_mlp* mlp, const uint16_t* feat_dev, int64_t n, float* logits_dev) {
  using namespace mlp;
  if (avs_status st = mlp_guard(mlp)) return st;
  if (!feat_dev || !logits_dev) return fail(AVS_E_INVALID, "null features or logits");
  if (n < 0 || n > INT32_MAX - TILE) return fail(AVS_E_INVALID, "n outside [0, 2^31 - 64]");
  if (n == 0) return AVS_OK;
  MCK(mlp_lds_attr());
  k_mlp_tile<FWD_LOGITS><<<(int)((n + TILE - 1) / TILE), TPB, LDS_BYTES, mlp->stream>>>(
      (int)n, feat_dev, nullptr, mlp->wbf, mlp->prm, logits_dev, nullptr, 0, nullptr, nullptr, 0.f, nullptr, nullptr);
  MCK(hipGetLastError());
  return AVS_OK;
}

avs_status avs_mlp_grad(avs_mlp* mlp, const uint16_t* feat_dev, const int8_t* flags_dev, const int32_t* rows_dev,
                        int64_t n, float* grad_dev, double* loss_host) {
  if (avs_status st = mlp_guard(mlp)) return st;
  if (avs_status st = mlp_check_batch(mlp, feat_dev, flags_dev, n)) return st;
  if (!grad_dev) return fail(AVS_E_INVALID, "grad_dev is null");
  if (avs_status st = mlp_grad_into(mlp, feat_dev, flags_dev, rows_dev, n, grad_dev)) return st;
  if (loss_host) {
    MCK(hipMemcpyAsync(loss_host, mlp->loss, sizeof(double), hipMemcpyDeviceToHost, mlp->stream));
    MCK(hipStreamSynchronize(mlp->stream));
  }
  return AVS_OK;
}

avs_status avs_mlp_adam(avs_mlp* mlp, const float* grad_dev, const avs_adam* hp) {
  if (avs_status st = mlp_guard(mlp)) return st;
  if (!grad_dev) return fail(AVS_E_INVALID, "grad_dev is null");
  if (avs_status st = mlp_check_adam(hp)) return st;
  return mlp_adam_launch(mlp, grad_dev, hp);
}

avs_status avs_mlp_train_step(avs_mlp* mlp, const uint16_t* feat_dev, const int8_t* flags_dev, const int32_t* rows_dev,
                              int64_t n, const avs_adam* hp, double* loss_host) {
  if (avs_status st = mlp_guard(mlp)) return st;
  if (avs_status st = mlp_check_batch(mlp, feat_dev, flags_dev, n)) return st;
  if (avs_status st = mlp_check_adam(hp)) return st;
  if (avs_status st = mlp_grad_into(mlp, feat_dev, flags_dev, rows_dev, n, mlp->grad)) return st;
  if (avs_status st = mlp_adam_launch(mlp, mlp->grad, hp)) return st;
  if (loss_host) {
    MCK(hipMemcpyAsync(loss_host, mlp->loss, sizeof(double), hipMemcpyDeviceToHost, mlp->stream));
    MCK(hipStreamSynchronize(mlp->stream));
  }
  return AVS_OK;
}

void avs_mlp_destroy(avs_mlp* mlp) { delete mlp; }

static avs_status launch_features(avs_ctx* ctx, const avs_mlp* mlp, uint16_t* feat) {
  using namespace mlp;
  const Leaves L = ctx->leaves(ctx->lcur);
  const double c_ref = std::sqrt(ctx->gas.R * mlp->T_ref);
  k_quantiles<<<24, TPB, 0, ctx->stream>>>(ctx->nc, ctx->W, ctx->gas.R, mlp->rho_ref, c_ref, mlp->T_ref, ctx->quant);
  CKL();
  k_features<<<(L.n + TPB - 1) / TPB, TPB, 0, ctx->stream>>>(L, ctx->base[0], ctx->base[1], ctx->lmax, ctx->quant, feat);
  CKL();
  return AVS_OK;
}

avs_status avs_features(avs_ctx* ctx, const avs_mlp* mlp, uint16_t* feat_dev) {
  if (avs_status st = guard(ctx)) return st;
  if (avs_status st = mlp_guard(mlp)) return st;
  if (ctx->D != 2) return fail(AVS_E_INVALID, "the learned proposal is defined for 2-D velocity spaces only");
  if (!feat_dev) return fail(AVS_E_INVALID, "feat_dev is null");
  return launch_features(ctx, mlp, feat_dev);
}

avs_status avs_adapt_learned(avs_ctx* ctx, avs_mlp* mlp, double C1, double C2, const double* probes_host,
                             int32_t nprobes, double tail_tol, int8_t* flags_dev, int64_t* n_new_host,
                             int32_t* fallback_host) {
  using namespace mlp;
  if (avs_status st = guard(ctx)) return st;
  if (avs_status st = mlp_guard(mlp)) return st;
  if (ctx->D != 2) return fail(AVS_E_INVALID, "the learned proposal is defined for 2-D velocity spaces only");
  if (std::isnan(C1) || std::isnan(C2)) return fail(AVS_E_INVALID, "C1/C2 must not be NaN");
  if (!(tail_tol >= 0)) return fail(AVS_E_INVALID, "tail_tol must be >= 0");
  if (avs_status st = upload_probes(ctx, probes_host, nprobes)) return st;
  if (mlp->stream != ctx->stream) MCK(hipStreamSynchronize(mlp->stream));
  ctx->plan_valid = false;
  const Leaves L = ctx->leaves(ctx->lcur);
  const int nb = (L.n + BLOCK - 1) / BLOCK;
  {
    ProfScope ps(ctx, K_LEARNED);
    if (avs_status st = launch_features(ctx, mlp, ctx->feat)) return st;
    CK(mlp_lds_attr());
    k_mlp_tile<FWD_FLAGS><<<(L.n + TILE - 1) / TILE, TPB, LDS_BYTES, ctx->stream>>>(
        L.n, ctx->feat, nullptr, mlp->wbf, mlp->prm, nullptr, L.level, ctx->lmax, ctx->raw, nullptr, 0.f, nullptr,
        nullptr);
    CKL();
    if (avs_status st = launch_sep_floor<2>(ctx, L)) return st;
    k_resolve<2><<<nb, BLOCK, 0, ctx->stream>>>(L, ctx->raw, ctx->eff, ctx->cnt);
    CKL();
    k_scan<<<1, BLOCK, 0, ctx->stream>>>(L.n, ctx->cnt, ctx->off);
    CKL();
  }
  bool fits = false;
  if (avs_status st = finish_plan(ctx, flags_dev, n_new_host, &fits)) return st;
  bool accept = false;
  if (fits) {
    // judge on the proposed leaves
    const int np = nprobes + 8;
    if (nprobes > 0)
      for (int p = 0; p < nprobes; ++p)
        CK(hipMemcpyAsync(ctx->tprobe + (size_t)p * 4, probes_host + (size_t)p * 4, sizeof(double) * 4,
                          hipMemcpyHostToDevice, ctx->stream));
    k_extremes<<<8, TPB, 0, ctx->stream>>>(ctx->nc, ctx->W, ctx->gas.R, ctx->tprobe + (size_t)nprobes * 4);
    CKL();
    k_tail<<<np, TPB, 0, ctx->stream>>>(ctx->leaves(ctx->lcur ^ 1), ctx->tprobe, ctx->gas.R, ctx->terr);
    CKL();
    std::vector<double> err(np);
    CK(hipMemcpyAsync(err.data(), ctx->terr, sizeof(double) * np, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    accept = true;
    for (int p = 0; p < np; ++p)
      if (!(err[p] <= tail_tol)) accept = false;
  }
  if (fallback_host) *fallback_host = accept ? 0 : 1;
  if (accept) return AVS_OK;
  ctx->plan_valid = false;
  if (avs_status st = DISPATCH(ctx, launch_adapt, ctx, C1, C2, nprobes)) return st;
  return finish_plan(ctx, flags_dev, n_new_host);
}

avs_status avs_set_separated(avs_ctx* ctx, double r_lo, double r_hi, int32_t level) {
  if (avs_status st = guard(ctx)) return st;
  if (level < 0) {
    ctx->sep_level = -1;
    return AVS_OK;
  }
  if (!(r_lo >= 0.0) || !(r_hi > r_lo) || !std::isfinite(r_hi))
    return fail(AVS_E_INVALID, "separated zone needs 0 <= r_lo < r_hi < inf");
  ctx->sep_lo = r_lo;
  ctx->sep_hi = r_hi;
  ctx->sep_level = level;
  return AVS_OK;
}

avs_status avs_auto_params(const avs_flow* flow, avs_auto* params_out, avs_vspace* vspace_out) {
  return auto_params_host(flow, params_out, vspace_out);
}

avs_status avs_initial_avs(avs_ctx* ctx, const avs_flow* flow, double C1, double C2, int64_t* n_leaves_host) {
  if (avs_status st = guard(ctx)) return st;
  if (std::isnan(C1) || std::isnan(C2)) return fail(AVS_E_INVALID, "C1/C2 must not be NaN");
  avs_auto a;
  avs_vspace vs;
  if (avs_status st = auto_params_host(flow, &a, &vs)) return st;
  const int D = ctx->D;
  bool same = flow->dim == D && vs.max_level == ctx->lmax && flow->R == ctx->gas.R;
  for (int d = 0; d < D; ++d)
    same = same && vs.base[d] == ctx->base[d] && vs.lo[d] == ctx->lo[d] && vs.hi[d] == ctx->hi[d];
  if (!same) return fail(AVS_E_INVALID, "the context's velocity space or gas constant is not the one avs_auto_params gives for this flow");
  // step 2: the box split L_w - 1 times (relative to the roots at level min(L_min, L_max))
  const int lr = std::min(a.L_min, a.L_max);
  const int lev = std::min(std::max(a.L_w - 1 - lr, 0), ctx->lmax);
  int64_t n = 1;
  int cnt[3] = {1, 1, 1};
  for (int d = 0; d < D; ++d) {
    cnt[d] = ctx->base[d] << lev;
    n *= cnt[d];
  }
  if (n > ctx->cap) return fail(AVS_E_CAPACITY, "uniform step-0 mesh of %" PRId64 " leaves exceeds leaf_capacity", n);
  std::vector<std::pair<uint64_t, int64_t>> order((size_t)n);
  std::vector<int> ix((size_t)n * D);
  for (int64_t k = 0; k < n; ++k) {
    int64_t r = k;
    for (int d = 0; d < D; ++d) {
      ix[(size_t)k * D + d] = (int)(r % cnt[d]);
      r /= cnt[d];
    }
    order[(size_t)k] = {morton(D, ctx->lmax, lev, &ix[(size_t)k * D]), k};
  }
  std::sort(order.begin(), order.end());
  std::vector<int32_t> lvl((size_t)n, lev), idx((size_t)n * D);
  for (int64_t j = 0; j < n; ++j)
    for (int d = 0; d < D; ++d) idx[(size_t)j * D + d] = ix[(size_t)order[(size_t)j].second * D + d];
  if (avs_status st = avs_set_leaves(ctx, n, lvl.data(), idx.data())) return st;
  // step 3: one adaptation over the freestream and static states only
  std::vector<double> probes(2 * (size_t)(D + 2), 0.0);
  probes[0] = flow->rho_inf;
  probes[D + 1] = flow->T_inf;
  probes[D + 2] = flow->rho_inf;
  probes[2 * (D + 2) - 1] = flow->T_inf;
  double norm = 0.0;
  for (int d = 0; d < D; ++d) norm += flow->direction[d] * flow->direction[d];
  norm = std::sqrt(norm);
  for (int d = 0; d < D; ++d) probes[1 + d] = norm > 0.0 ? a.U_inf * (flow->direction[d] / norm) : 0.0;
  if (avs_status st = upload_probes(ctx, probes.data(), 2)) return st;
  // the separated zone: 3 sigma_w < |xi| < 5 sigma_w at L_sep, for this and
  // every later adaptation (the flow decides: cleared when it does not separate)
  if (flow->separated) {
    ctx->sep_lo = 3.0 * a.sigma_w;
    ctx->sep_hi = 5.0 * a.sigma_w;
    ctx->sep_level = a.L_sep - lr;
  } else {
    ctx->sep_level = -1;
  }
  ctx->plan_valid = false;
  if (avs_status st = DISPATCH(ctx, launch_adapt, ctx, C1, C2, 2, false)) return st;
  int64_t n_new = 0;
  if (avs_status st = finish_plan(ctx, nullptr, &n_new)) return st;
  // commit the new leaves, then the conservative discrete Maxwellian of W on them
  if (avs_status st = avs_remap(ctx, 0)) return st;
  if (avs_status st = DISPATCH(ctx, launch_init_vdf, ctx)) return st;
  if (avs_status st = DISPATCH(ctx, launch_moments, ctx)) return st;
  if (avs_status st = check_bad(ctx)) return st;
  if (n_leaves_host) *n_leaves_host = n_new;
  return AVS_OK;
}

void avs_destroy(avs_ctx* ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
  delete ctx;
}

const char* avs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
