/*
 * avs.h -- C ABI of the MI355X (gfx950) global adaptive-velocity-space sweep.
 *
 * The library advances the reduced distribution functions (G, H in 2-D; G in
 * 3-D) of a monatomic gas on ONE velocity mesh shared by every physical cell
 * (the paper's "global velocity mesh", Sec. 1 and Sec. 3), over a
 * finite-volume physical mesh, and adapts that velocity mesh with the
 * quadtree/octree split/merge rules of Sec. 3.
 *
 * Paper: J. Chen, S. Liu, R. Zhang, C. Zhong, Y. Yang, C. Zhuo, "A global
 * adaptive velocity space for general discrete velocity framework in
 * predictions of rarefied and multi-scale flows", arXiv:2212.05645.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  The library never allocates device memory.  The caller provides
 *   two device regions at init: the VDF region (size avs_vdf_bytes: the
 *   current and next VDF plus one interface row per face) and a workspace
 *   (size avs_workspace_bytes); both must stay alive and untouched by the
 *   caller until avs_destroy.  Arguments named *_host are host
 *   pointers, *_dev device pointers.
 * Layout.  VDF values are stored component-major, cell-major, leaf-fastest:
 *   vdf[comp][cell][leaf] with a row stride of avs_leaves().ld elements.
 *   Leaves are kept in depth-first (Morton) order of the velocity forest.
 *   Conserved variables W = (rho, rho U_1..U_D, rho E) (Eq. updat_W);
 *   primitive rows are (rho, U_1..U_D, T).
 * Streams.  All device work is enqueued on the stream given at init
 *   (a hipStream_t passed as void*, NULL = default stream).  A call waits for
 *   the device only when it returns a *_host output or says so below.
 * Errors.  Arguments are validated before any device work.  On a non-OK
 *   return the state is unchanged, except AVS_E_HIP and AVS_E_NUMERIC found
 *   after device work, which leave the context in the failed state
 *   (AVS_E_STATE on every later call except avs_destroy / avs_last_error).
 *   avs_last_error() returns a message for the calling thread's last error.
 * Threads.  A context is not thread-safe; separate contexts are independent.
 * Units.  Non-dimensional; the gas constant R is a parameter.
 */
#ifndef AVS_H
#define AVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t avs_status;
#define AVS_OK 0
#define AVS_E_INVALID (-1)   /* bad argument or unsupported mesh */
#define AVS_E_CAPACITY (-2)  /* the adapted velocity mesh would exceed leaf_capacity */
#define AVS_E_HIP (-3)       /* a HIP runtime call failed */
#define AVS_E_STATE (-4)     /* call not valid in the current state */
#define AVS_E_NUMERIC (-5)   /* non-positive density/temperature or singular moment system */

#define AVS_BC_WALL 0        /* isothermal, fully diffuse wall (zero net mass flux) */
#define AVS_BC_FARFIELD 1    /* incoming molecules from the far-field Maxwellian */

#define AVS_FP64 0
#define AVS_FP32 1

#define AVS_COPY 0
#define AVS_SPLIT 1
#define AVS_MERGE 2

typedef struct avs_ctx avs_ctx;

/* Velocity space: a forest of base[0] x base[1] (x base[2]) level-0 roots on
 * the box [lo, hi] (Sec. 3.1); each root may be split down max_level levels.
 * leaf_capacity bounds the number of leaves any adaptation may produce. */
typedef struct {
  int32_t dim;             /* 2 or 3 */
  int32_t max_level;       /* 0..12 */
  int32_t base[3];         /* roots per axis, >= 1 */
  double lo[3], hi[3];     /* velocity box */
  int64_t leaf_capacity;   /* >= number of roots */
} avs_vspace;

/* Gas model (Sec. 2.1-2.2): relaxation time tau = mu(T) / (rho R T) (Eq.
 * equ3) with mu(T) = mu_ref (T/T_ref)^omega (law 0, VHS power law) or
 * mu_ref (T/T_ref)^(3/2) (T_ref + C_s)/(T + C_s) (law 1, Sutherland, Eq.
 * Sutherland of Sec. 4.6; C_s >= 0 in the units of T); model 0 = BGK
 * target, 1 = Shakhov target with Prandtl number Pr (Eqs. equ14-equ17). */
typedef struct {
  double R, Pr, omega, mu_ref, T_ref;
  int32_t model;
  int32_t law;     /* 0 power law, 1 Sutherland */
  double C_s;      /* Sutherland constant (law 1) */
} avs_gas;

/* Finite-volume mesh, host arrays, copied at init.  face_lr[f] = (L, R); a
 * boundary face has R = -1 - bc_id and its normal points out of L.  Normals
 * are unit vectors from L to R.  face_shift (may be NULL) is added to the
 * centre of R to place it next to L across a periodic seam.  Every cell may
 * have at most 4 faces in 2-D and 6 in 3-D.  bc_state rows are primitive
 * (rho, U, T); rho is ignored for walls. */
typedef struct {
  int32_t dim;
  int64_t ncells, nfaces;
  const double *cell_vol;   /* [ncells] */
  const double *cell_ctr;   /* [ncells][dim] */
  const int64_t *face_lr;   /* [nfaces][2] */
  const double *face_area;  /* [nfaces] */
  const double *face_nrm;   /* [nfaces][dim] */
  const double *face_ctr;   /* [nfaces][dim] */
  const double *face_shift; /* [nfaces][dim] or NULL */
  int32_t nbc;
  const int32_t *bc_kind;   /* [nbc] AVS_BC_* */
  const double *bc_state;   /* [nbc][dim+2] */
} avs_pmesh;

/* Numerical options.  dt > 0 is the time step; venkat_K the constant of the
 * Venkatakrishnan limiter, eps^2 = (K V^(1/D))^3.  precision selects the VDF
 * storage/flux type (AVS_FP64, or AVS_FP32 with FP64 conserved variables). */
typedef struct {
  int32_t precision;
  double dt;
  double venkat_K;
} avs_opts;

/* Reference viscosity for a Knudsen number Kn = lambda / L_ref at the state
 * (rho_ref, T_ref) (Eqs. equ4, equ5). */
double avs_mu_ref_from_kn(double Kn, double omega, double R, double T_ref, double rho_ref, double L_ref);

/* Bytes the caller must provide for the VDF region / the workspace. */
size_t avs_vdf_bytes(const avs_vspace *vs, const avs_pmesh *pm, const avs_opts *op);
size_t avs_workspace_bytes(const avs_vspace *vs, const avs_pmesh *pm, const avs_opts *op);

/* Create a context on the level-0 forest and set phi = closure(g_eq(W0), W0)
 * per cell, with W0 built from prim0_host [ncells][dim+2]: the initial
 * distribution is the Maxwellian of Eq. Maxwell_df (in 2-D the reduced pair
 * G and H = (3 - D) R T G) of each cell's initial state, as Sec. 3.5
 * starts the adaptive run, sampled at the leaf centres and corrected so that
 * its discrete moments equal W0 (the conservation correction of Sec. 3.3).  Copies every host array; waits for
 * the device before returning.  The descriptors, the mesh (face ranges, at
 * most 4 / 6 faces per cell, areas, volumes) and the initial states are
 * checked on the host, and the per-cell tables built there, before any HIP
 * call: those errors are AVS_E_INVALID with no device work done. */
avs_status avs_init_mesh(const avs_vspace *vs, const avs_pmesh *pm, const avs_gas *gas, const avs_opts *op,
                         const double *prim0_host, void *vdf_dev, size_t vdf_bytes, void *workspace_dev,
                         size_t workspace_bytes, void *hip_stream, avs_ctx **out);

/* Advance nsteps explicit steps (Sec. 2.3 with the implicit flux increments
 * dropped): upwind limited reconstruction at x_f - xi h, interface
 * moments and Shakhov equilibrium, interface VDF of Eq. equ28, finite-volume
 * update of W (Eq. equ18), relaxation of every node towards the
 * moment-closed Shakhov target.  h = dt/2, capped at half of the largest
 * step for which no cell's outflow over the velocity box exceeds its
 * content (min_i V_i / (1/2 sum_f A_f sum_d |n_fd| max(|lo_d|, |hi_d|))),
 * so that x_f - xi h stays within reach of the upwind cell (Sec. 2.3.3);
 * the cap only binds for steps beyond that explicit bound.  residual_host (or NULL) receives
 * |W^{n+1} - W^n|_2 / dt per conserved component for the last step; a
 * non-NULL residual makes the call wait and report AVS_E_NUMERIC if any cell
 * went non-physical. */
avs_status avs_step(avs_ctx *ctx, int32_t nsteps, double *residual_host);

/* Wait for the context's stream and report what the kernels found since the
 * context was made: AVS_E_NUMERIC (and the failed state) if some cell's
 * state became non-physical or its moment system singular, or some
 * interface state non-physical.  avs_step reports this only when it
 * returns a residual; avs_remap always does.  Use it after steps timed
 * without a residual. */
avs_status avs_check(avs_ctx *ctx);

/* Rykov model constants of a diatomic gas (Sec. 2.2; nitrogen: delta =
 * 1/1.55, omega_0 = 0.2354, omega_1 = 0.3049); Z_rot, the rotational
 * collision number, is the gas's (the paper gives no value). */
typedef struct {
  double Z_rot, delta, omega0, omega1;
} avs_rykov;

/* Rykov equilibrium of the diatomic model (Eqs. GHR_equ, equ11-equ13) on the
 * context's current leaves: for each of n states, g^phi = (1 - 1/Z_rot)
 * phi^t + (1/Z_rot) phi^r for phi = G, H (the 3 - D hidden translational
 * degrees of freedom, zero in 3-D) and R (rotational energy, two degrees of
 * freedom), with T = (3 T_t + 2 T_r)/5, p_t = rho R T_t, p = rho R T and the
 * context's gas constant R.  states_dev: device array [n][3 + 3D] of
 * (rho, U[D], T_t, T_r, q_t[D], q_r[D]) in FP64, read only.  out_dev:
 * device array [3][n][ld] (ld = the row stride avs_leaves reports) in the
 * context's precision, written for the first nleaves entries of each row;
 * out_bytes >= 3 n ld element size, else AVS_E_INVALID.  Asynchronous on the
 * context's stream.  A building block of the diatomic model: the sweep of
 * avs_step is monatomic. */
avs_status avs_rykov_equilibrium(avs_ctx *ctx, const avs_rykov *gas, const double *states_dev, int64_t n,
                                 void *out_dev, size_t out_bytes);

/* Explicit steps of the Rykov diatomic model on a context's mesh and current
 * leaves: FP64 contexts, 2-D or 3-D.  Three reduced distributions G, H, R
 * (Eq. equ6; H is the 3 - D hidden translational degrees of freedom, zero
 * in 3-D) and W = (rho, rho U, rho E, rho E_rot) (Eq. updat_W).
 * One step: limited upwind reconstruction at x_f - xi h (h as in avs_step);
 * interface moments, the rotational energy relaxed over h towards rho R T
 * (the relation after Eq. w_interface, read with its factor as a divisor)
 * and heat fluxes relaxed at the rates the Rykov equilibrium gives them;
 * the interface VDF of Eq. equ28 with the Rykov equilibrium (Eqs. GHR_equ,
 * equ11-equ13); W* = W - dt/V sum A F and the rotational exchange of Eq.
 * equ19, point-implicit with tau = mu(T_t)/p_t of W*; relaxation of G, H, R
 * towards the Rykov equilibrium of W^{n+1} closed onto (rho, rho U, rho E,
 * (1 - 1/Z) rho E_rot + rho R T / Z).  Walls and far field take equilibrium
 * triples (g, R T g, R T g) of their state; the wall's density gives zero net
 * mass flux.  The state lives in a caller region of avs_dia_bytes bytes
 * (device, 256-byte aligned, owned by the caller until avs_dia_destroy),
 * sized for at most max_leaves leaves (between the current leaf count and
 * the context's leaf capacity).
 * prim0_host: [ncells][D+3] = (rho, U, T_t, T_r); the initial VDF is
 * the translational part of the Rykov equilibrium at (T_t, T_r) closed onto
 * W.  The context's leaves may change only through avs_dia_remap while the
 * state is used (AVS_E_STATE otherwise); the monatomic state of the context
 * is not otherwise touched.  avs_dia_step waits for the device and reports AVS_E_NUMERIC for
 * a non-physical state.  avs_dia_get_state copies [3][ncells][nleaves] and
 * [ncells][D+3] (either may be NULL). */
typedef struct avs_dia avs_dia;
avs_status avs_dia_bytes(const avs_ctx *ctx, int64_t max_leaves, size_t *bytes);
avs_status avs_dia_create(avs_ctx *ctx, const avs_rykov *gas, const double *prim0_host, int64_t max_leaves,
                          void *mem_dev, size_t mem_bytes, avs_dia **out);
avs_status avs_dia_step(avs_dia *dia, int32_t nsteps);
avs_status avs_dia_get_state(avs_dia *dia, double *vdf_host, double *W_host);

/* Implicit steps of the diatomic model (Secs. 2.3.1-2.3.2 with the
 * rotational row of Eqs. S_rot and SGS_wrot), at the context's dt.  As
 * avs_step_implicit, with the interface stage above, and:
 *  - predictor over the D + 3 variables: the Euler flux carries
 *    rho E_rot U.n and uses the translational pressure rho R T_t, so r_f
 *    takes the frozen sound speed sqrt(5/3 R T_t) and mu/rho = tau R T_t;
 *  - the rotational row's diagonal and right-hand side gain V/(Z tau) and
 *    V (rho R T - rho E_rot^n)/(Z tau), at the cell's current iterate;
 *  - W^{n+1} in flux form with the implicit flux, then the rotational
 *    exchange, target and tau~ as in avs_dia_step;
 *  - n_micro symmetric Gauss-Seidel sweeps over G, H, R.
 * No memory beyond the state's region: the micro right-hand side and
 * increment use the spare state and interface buffers (the mesh needs
 * ncells <= nfaces + 1, AVS_E_INVALID otherwise).  n_macro = n_micro = 0 is
 * allowed (zero increments).  Waits for the device; AVS_E_NUMERIC for a
 * non-physical state. */
avs_status avs_dia_step_implicit(avs_dia *dia, int32_t nsteps, int32_t n_macro, int32_t n_micro);

/* Adaptation of the velocity tree driven by the diatomic state (Secs.
 * 3.2-3.4): M_k = max over cells of max(M1, M2), M1 = A G / rho, M2 =
 * A (1/2 (|c|^2 G + H) + R) / (rho E - rho |U|^2 / 2) (the internal energy
 * includes rotation), over the cells and over the nprobes probe states:
 * rows (rho, U, T) [nprobes][D+2] of equilibrium states (T_t = T_r = T)
 * whose VDF is the equilibrium triple (g, (3 - D) R T g, R T g), internal
 * energy 5/2 rho R T (at most the context's probe capacity; NULL with 0).
 * Flags and plan as avs_adapt.
 * flags_dev and n_new_host as in avs_adapt; AVS_E_CAPACITY (plan discarded)
 * beyond the state's max_leaves or the context's capacity.
 * avs_dia_remap applies the plan: consanguinity reconstruction of G, H, R
 * and the closure onto W, the heat fluxes of the result, and avs_remap(ctx,
 * 0) for the context's own state, which moves the context to the new
 * leaves; the diatomic state follows them. */
avs_status avs_dia_adapt(avs_dia *dia, double C1, double C2, const double *probes_host, int32_t nprobes,
                         int8_t *flags_dev, int64_t *n_new_host);
avs_status avs_dia_remap(avs_dia *dia);
void avs_dia_destroy(avs_dia *dia);

/* Bytes of the device region avs_step_implicit needs for the right-hand
 * side of the micro system: one VDF buffer (components x cells x leaf
 * capacity x element size). */
avs_status avs_implicit_bytes(const avs_ctx *ctx, size_t *bytes);

/* Advance nsteps implicit steps (IUGKS, Sec. 2.3.1-2.3.2) with the context's
 * dt (no explicit stability bound applies to it).  Interface VDFs and
 * fluxes F^n as in avs_step; then the macroscopic predictor of Eqs.
 * equ_delw, delta_Flux, Roe and SGS_w (Roe-type flux increment with
 * r = |U.n| + a + 2 mu/(rho dl) from the interface state, a boundary face
 * holding the outside increment at zero) solved by macro_sweeps symmetric
 * point-relaxation Gauss-Seidel sweeps; the closed Shakhov target and tau
 * from W^{n+1}; the upwind micro system of Eq. SGS_phi solved by
 * micro_sweeps symmetric Gauss-Seidel sweeps; phi^{n+1} = phi^n + dphi.
 * W^{n+1} takes the flux form of Eq. equ18 with the Roe-type implicit flux
 * of the predicted increment on interior faces and the explicit flux on
 * boundary faces (exactly conservative after any number of sweeps, no
 * increment through walls, the predicted W on a periodic mesh once the
 * sweeps converge), and the target and tau are built from it.  The interface half step is min(dt/2, the cap of avs_step)
 * whatever dt is.  Each sweep runs the colours of a greedy
 * colouring of the cells in cell order (smallest colour no lower-numbered
 * face neighbour holds) up, then down; the paper recommends 60 macro and 2
 * micro sweeps.  res_dev: device scratch of avs_implicit_bytes bytes,
 * 256-byte aligned, owned by the caller, overwritten.  residual_host as in
 * avs_step.  Waits for the device; AVS_E_NUMERIC if a predicted state is
 * non-physical, AVS_E_INVALID for negative counts or a short region. */
avs_status avs_step_implicit(avs_ctx *ctx, int32_t nsteps, int32_t macro_sweeps, int32_t micro_sweeps, void *res_dev,
                             size_t res_bytes, double *residual_host);

/* Per-cell fields (rho, U_1..U_D, T, q_1..q_D) into fields_dev
 * [ncells][2*dim+2] (rho, U, T from the authoritative W; q = heat flux of the
 * VDF about U, Eq. equ8) and/or the FP64 totals sum_i V_i W_i into
 * totals_host [dim+2] (waits).  Either pointer may be NULL. */
avs_status avs_moments(avs_ctx *ctx, double *fields_dev, double *totals_host);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * outputs as avs_moments, with the partial sums of the totals in a static
 * device array of the library (5 125 doubles, about 40 KiB per device, held
 * until the process ends) instead of the context's workspace.  It calls no
 * allocating routine.  Limit: at most 1 048 576 cells when totals_host is
 * non-NULL, else AVS_E_CAPACITY before any device work; AVS_E_HIP if the
 * array has no address on the context's device.  All calls on one device
 * share the array: calls that overlap on one device (other streams or
 * threads) race; calls in order on one stream do not.  Totals agree with
 * avs_moments to rounding (another summation order); fields bit for bit. */
avs_status avs_moments_noalloc(avs_ctx *ctx, double *fields_dev, double *totals_host);

/* Adaptation (Sec. 3.4): M_k = max over cells (and over the nprobes probe
 * states, primitive rows whose VDF is the discrete Maxwellian) of
 * max(M1, M2) (Eqs. criterion_rho, criterion_e, criterion_mk); split if
 * M_k > C1 below max_level, merge a full brother group if all its members
 * have M_k < C2 (Sec. 3.1), keep otherwise.  Builds the new leaf list and
 * the remap plan on the device.  flags_dev (or NULL) receives the effective
 * flag per current leaf (-1 merge, 0 keep, +1 split).  Waits; *n_new_host
 * gets the new leaf count.  Returns AVS_E_CAPACITY (plan discarded) if it
 * exceeds leaf_capacity. */
avs_status avs_adapt(avs_ctx *ctx, double C1, double C2, const double *probes_host, int32_t nprobes,
                     int8_t *flags_dev, int64_t *n_new_host);

/* Apply the plan of the last avs_adapt: consanguinity remap (Sec. 3.2; a
 * child copies its parent, a merged parent is the pairwise mean of its
 * children), then correction 0 = none, 1 = f' + g_eq(W) - g_eq(W') (Sec. 3.3),
 * 2 = that plus the closure that restores M[f] = W to round-off.
 * correction 3 = the equilibrium bypass for weakly non-equilibrium flow (end
 * of Sec. 3.3): the new leaves take the discrete Maxwellian g_eq(W) of each
 * cell's W (H = (3 - D) R T G) and the old distribution is not read, so mass,
 * momentum and energy hold only to quadrature error; 4 = that Maxwellian
 * closed onto W like the initial state.  Other values: AVS_E_INVALID. */
avs_status avs_remap(avs_ctx *ctx, int32_t correction);

/* Current velocity mesh.  *n_host = leaf count, *ld_host = VDF row stride.
 * Optional outputs (NULL to skip), host arrays of n entries: level, index at
 * that level ([n][dim]), centre ([n][dim]) and weight (area/volume). */
avs_status avs_leaves(avs_ctx *ctx, int64_t *n_host, int64_t *ld_host, int32_t *level_host, int32_t *idx_host,
                      double *xi_host, double *w_host);

/* Remap plan of the last avs_adapt (host arrays of n_new entries). */
avs_status avs_plan(avs_ctx *ctx, int32_t *kind_host, int64_t *src_host, int32_t *child_host);

/* M_k of the last avs_adapt, [n_old] host doubles. */
avs_status avs_criterion(avs_ctx *ctx, double *Mk_host);

/* Replace the velocity mesh by the given leaves (host, depth-first order,
 * validated) and reset phi = closure(g_eq(W), W) from the current W. */
avs_status avs_set_leaves(avs_ctx *ctx, int64_t n, const int32_t *level_host, const int32_t *idx_host);

/* Copy the state out / in.  vdf_host is [P][ncells][n] FP64 (P = 2 in 2-D,
 * 1 in 3-D; converted from/to the storage type), W_host is [ncells][dim+2].
 * avs_set_state with vdf_host == NULL sets phi = closure(g_eq(W), W); with
 * W_host == NULL it sets W to the moments of the given VDF (Eq. updat_W,
 * AVS_E_NUMERIC if they are not physical).  Either pointer of avs_get_state
 * may be NULL.  Both wait. */
avs_status avs_get_state(avs_ctx *ctx, double *vdf_host, double *W_host);
avs_status avs_set_state(avs_ctx *ctx, const double *vdf_host, const double *W_host);

/* VDF rows of selected cells, [P][ncell_sel][n] FP64 host (waits). */
avs_status avs_get_cells(avs_ctx *ctx, int64_t ncell_sel, const int64_t *cells_host, double *vdf_host);

/* Measurement support (not part of the method).  avs_profile(ctx, 1) waits
 * for the stream, clears earlier records and brackets every subsequent kernel
 * group of the context with a pair of HIP events on its stream; 0 stops.
 * avs_profile_read waits and writes, for at most nmax kernel groups that ran,
 * a name (32 chars per entry in names_host), the summed milliseconds and the
 * number of launches; it returns the number of entries or -1 on error. */
avs_status avs_profile(avs_ctx *ctx, int32_t enable);
int32_t avs_profile_read(avs_ctx *ctx, int32_t nmax, char *names_host, double *ms_host, int64_t *count_host);

/* Batched form: many independent contexts (same dimension, precision and
 * non-default stream) advance in the same launches -- one launch per step
 * kernel covers the workgroups of every case -- and avs_batch_step with
 * use_graph != 0 captures the whole nsteps sequence in one HIP graph that
 * is replayed until a case's leaf count or the tile choice changes.  The
 * members stay usable on their own (adapt, remap, moments) between batch
 * steps.  The batch workspace (device, avs_batch_workspace_bytes) holds the
 * per-case argument tables.  avs_batch_tune chooses two tile parameters
 * by timing: the leaf chunk of pass A (512..16384 leaves per workgroup) per
 * leaf-count bucket of the members (< 1024, < 4096, < 16384, more leaves),
 * one bucket at a time, then whether pass C keeps one or two leaves' loads
 * in flight; each candidate is timed on two steps computed into the spare
 * buffers and not taken, so the members' state is the same afterwards
 * (their implicit-predictor and remap scratch is overwritten).  chunk_host
 * (or NULL) receives five ints: the four chunks and the pass-C choice (0/1).
 * avs_batch_check waits and reports a non-physical state in any member. */
typedef struct avs_batch avs_batch;
size_t avs_batch_workspace_bytes(int32_t ncase);
avs_status avs_batch_create(int32_t ncase, avs_ctx *const *ctxs, void *workspace_dev, size_t workspace_bytes,
                            avs_batch **out);
avs_status avs_batch_step(avs_batch *batch, int32_t nsteps, int32_t use_graph);
avs_status avs_batch_check(avs_batch *batch);
avs_status avs_batch_tune(avs_batch *batch, int32_t *chunk_host);
/* avs_adapt (no probe states, no flags) for every member, case i with
 * thresholds C1_host[i], C2_host[i]: the criterion, flags and scan of all
 * cases are enqueued on four side streams (forked from and joined back to
 * the batch's stream), the new leaf counts (n_new_host[i], or NULL) are read
 * with one wait, then every new leaf list and remap plan is built.
 * AVS_E_CAPACITY names the first case over its leaf_capacity; no plan is
 * then valid.  avs_batch_remap applies avs_remap(correction) to every member
 * (corrections 0-2 as launches spanning all members, 3-4 per member) and
 * reports a non-physical state in any of them.  Results are those of the
 * per-case calls, bit for bit.  Both wait for the device. */
avs_status avs_batch_adapt(avs_batch *batch, const double *C1_host, const double *C2_host, int64_t *n_new_host);
avs_status avs_batch_remap(avs_batch *batch, int32_t correction);
void avs_batch_destroy(avs_batch *batch);

/* Learned refinement proposal (not part of the paper; 2-D only).  A network
 * predicts, for every leaf, the decision of the criterion of Sec. 3.4 after
 * the brother-group rule of Sec. 3.1 (class 0 keep, 1 split, 2 merge) from
 * 28 features: the leaf centre relative to the box centre over the box
 * half-width (2), its width over the box width (1), level / max_level (1),
 * and the lower quantiles at 0, 1/5, .., 1 (element j (ncells-1)/5 of the
 * sorted values) of rho/rho_ref, U_x/sqrt(R T_ref), U_y/sqrt(R T_ref) and
 * T/T_ref over the cells (24).  Network 28 -> 128 -> 128 -> 3, ReLU; inputs,
 * weights and hidden activations in bfloat16 (nearest, ties to even), MFMA
 * products accumulated in float32, biases and logits float32.  Training
 * minimises the mean softmax cross-entropy with Adam; the backward deltas
 * are rounded to bfloat16 where the forward rounds.
 *
 * Parameters: one float32 vector of avs_mlp_param_count() = 20611 values,
 * W1 [28][128], b1 [128], W2 [128][128], b2 [128], W3 [128][3], b3 [3]
 * (row-major, input index first).  The network's device state (parameters,
 * Adam moments, bfloat16 weights, per-tile gradients for batches of up to
 * max_batch samples) lives in caller memory of avs_mlp_state_bytes(max_batch)
 * bytes; all its work runs on the stream given at creation.  Feature rows
 * are bfloat16 [n][32] (28 used, the rest zero); labels are effective flags
 * (-1 merge, 0 keep, +1 split) as avs_adapt writes them; rows_dev (int32
 * [n], or NULL for 0..n-1) selects the dataset rows of a batch: every entry
 * must index a row that exists in feat_dev and flags_dev (device data, not
 * checked). */
typedef struct avs_mlp avs_mlp;
typedef struct {
  double lr, beta1, beta2, eps;   /* Adam (Kingma and Ba, 2015) */
} avs_adam;
int64_t avs_mlp_param_count(void);
size_t avs_mlp_state_bytes(int64_t max_batch);
/* Copies params_host [20611]; rho_ref, T_ref normalise the field features. */
avs_status avs_mlp_create(const float *params_host, int64_t max_batch, double rho_ref, double T_ref, void *state_dev,
                          size_t state_bytes, void *hip_stream, avs_mlp **out);
/* Parameters out / in (waits); set also clears the Adam moments and step. */
avs_status avs_mlp_get_params(avs_mlp *mlp, float *params_host);
avs_status avs_mlp_set_params(avs_mlp *mlp, const float *params_host);
/* Logits [n][3] float32 of the feature rows (n <= max_batch not required). */
avs_status avs_mlp_forward(avs_mlp *mlp, const uint16_t *feat_dev, int64_t n, float *logits_dev);
/* Mean loss (loss_host, waits; NULL to skip) and its gradient grad_dev
 * [20611] float32 over a batch of n <= max_batch rows. */
avs_status avs_mlp_grad(avs_mlp *mlp, const uint16_t *feat_dev, const int8_t *flags_dev, const int32_t *rows_dev,
                        int64_t n, float *grad_dev, double *loss_host);
/* One Adam step with a given gradient grad_dev [20611]. */
avs_status avs_mlp_adam(avs_mlp *mlp, const float *grad_dev, const avs_adam *hp);
/* avs_mlp_grad into the state's own buffer, then avs_mlp_adam. */
avs_status avs_mlp_train_step(avs_mlp *mlp, const uint16_t *feat_dev, const int8_t *flags_dev, const int32_t *rows_dev,
                              int64_t n, const avs_adam *hp, double *loss_host);
void avs_mlp_destroy(avs_mlp *mlp);

/* Feature rows of the context's current leaves into feat_dev [nleaves][32]
 * (enqueued on the context's stream). */
avs_status avs_features(avs_ctx *ctx, const avs_mlp *mlp, uint16_t *feat_dev);

/* Adaptation with the learned proposal: features, network, arg max (lowest
 * class on ties; split only below max_level, merge only above the roots),
 * the brother-group rule, the new leaf list and remap plan.  Judge: for each
 * probe state (the nprobes given primitive rows, then the cells holding the
 * minimum and the maximum of rho, U_x, U_y and T, lowest index on ties) the
 * relative error of the discrete density and energy of its Maxwellian on the
 * proposed leaves must not exceed tail_tol; otherwise, or if the proposal
 * would exceed leaf_capacity, the plain criterion (avs_adapt with C1, C2 and
 * the same probes) decides.  *fallback_host = 1 when it did.  Outputs and
 * errors as avs_adapt; waits for the network's stream first. */
avs_status avs_adapt_learned(avs_ctx *ctx, avs_mlp *mlp, double C1, double C2, const double *probes_host,
                             int32_t nprobes, double tail_tol, int8_t *flags_dev, int64_t *n_new_host,
                             int32_t *fallback_host);

/* ---- Automatic velocity space (Sec. 3.5) -------------------------------
 * The adaptive parameters of Sec. 3.5 from the freestream, and the step-0
 * velocity space.  Host computation, except for the adaptation of
 * avs_initial_avs, which runs on the context's stream. */
typedef struct {
  int32_t dim;            /* 2 or 3 */
  double R, gamma;        /* gas constant (solver units) and ratio of specific heats, > 0 and > 1 */
  double Ma;              /* freestream Mach number, >= 0 */
  double T_inf, T_wall;   /* freestream static and wall temperatures, > 0 */
  double rho_inf;         /* freestream density, > 0 */
  double direction[3];    /* freestream direction, normalised here; non-zero when Ma > 0 */
  double rdv_sigmas;      /* R_dv in units of sigma_0 (> 0; the paper uses 4, up to 7 for hot walls) */
  double h_std;           /* standard velocity interval (> 0; the paper uses 0.6) */
  int32_t separated;      /* non-zero: the flow separates, and avs_initial_avs refines the separated zone */
} avs_flow;

typedef struct {
  double T0;                            /* total temperature, Eq. totaltemperature */
  double sigma_inf, sigma_0, sigma_w;   /* sqrt(R T) of T_inf, T0, T_wall */
  double U_inf;                         /* Ma sqrt(gamma R T_inf) */
  double centre[3], R_dv;               /* box centre 0.4 U_inf e and half-width rdv_sigmas sigma_0 */
  double h_min;                         /* 2 R_dv / 2^L_max */
  int32_t L_max;                        /* smallest L with 2^L >= 2 R_dv / h_std */
  int32_t L_w;                          /* L_max, or L_max - 1 when T_wall / T_inf >= 4 */
  int32_t L_min;                        /* 4 for dim 2 and Ma > 5, else 3 */
  int32_t L_sep;                        /* separated zone, max(L_min, L_w - 1) */
  double C1, C2, k_sigma;               /* 13.749 Ma^-1.465 (Eq. C1_Ma), k_sigma C1, k_sigma = e^-8 (Eq. c2c1) */
} avs_auto;

/* Parameters of Sec. 3.5 for flow, and the velocity space that realises
 * them on the solver's forest: 2^min(L_min, L_max) roots per axis on the box
 * centre -/+ R_dv, L_max - min(L_min, L_max) levels below them, and
 * leaf_capacity = leaves of the complete tree (at most 2^26).  Either output
 * may be NULL.  AVS_E_INVALID for out-of-range inputs or a box that needs
 * more levels than the solver supports. */
avs_status avs_auto_params(const avs_flow *flow, avs_auto *params_out, avs_vspace *vspace_out);

/* Step-0 velocity space (Sec. 3.5, steps 1-3) on a context created with the
 * avs_vspace that avs_auto_params returned for flow (checked): the uniform
 * mesh after L_w - 1 splits of the box (the roots when that is fewer than
 * their level), one adaptation whose criterion runs over the freestream
 * (rho_inf, U_inf e, T_inf) and the static state (rho_inf, 0, T_inf) only,
 * with thresholds C1, C2 (the fit of Eq. C1_Ma is far above every M_k of
 * the criterion as printed, so the caller chooses them), then phi =
 * closure(g_eq(W), W) on the new leaves for the current W.  Writes the leaf
 * count to *n_leaves_host (may be NULL).  Waits for the device. */
avs_status avs_initial_avs(avs_ctx *ctx, const avs_flow *flow, double C1, double C2, int64_t *n_leaves_host);
/* With flow->separated non-zero, avs_initial_avs first installs the
 * separated zone of Sec. 3.5, avs_set_separated(ctx, 3 sigma_w, 5 sigma_w,
 * L_sep - min(L_min, L_max)), which then holds for its adaptation and every
 * later one on the context; with it zero, it clears any zone. */

/* Separated zone (Sec. 3.5): a floor on the flags of every later adaptation
 * of the context (avs_adapt, avs_adapt_learned, the batched and diatomic
 * adaptations).  An element whose discrete velocity (its centre) lies in
 * the open annulus r_lo < |xi| < r_hi about the origin keeps at least
 * `level`, counted from the forest's roots: such a leaf below it is flagged
 * to split (below max_level), and a merge whose parent would be centred
 * there below it does not happen.  Radii are compared squared, |xi|^2
 * summed axis by axis in FP64.  level < 0 removes the zone.  Host only;
 * AVS_E_INVALID unless 0 <= r_lo < r_hi < inf. */
avs_status avs_set_separated(avs_ctx *ctx, double r_lo, double r_hi, int32_t level);

/* Release the context (never frees caller memory). */
void avs_destroy(avs_ctx *ctx);

/* Message of the calling thread's last error ("" if none). */
const char *avs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AVS_H */
