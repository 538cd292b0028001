/*
 * acopf.h -- C ABI of the MI355X (gfx950) ACOPF model-evaluation library.
 *
 * The library evaluates the ACOPF model at an interior-point iterate, the
 * work an interior-point solver repeats every iteration (paper: OPFLOW
 * section, compact statement min f(x) s.t. g(x) = 0, h- <= h(x) <= h+,
 * x- <= x <= x+, evaluated on the GPU with the data kept resident there).
 * What follows describes the power-balance-polar form without slack
 * variables, which acopf_net_create builds; the cartesian form and the
 * feasibility slacks (acopf_net_create_opts) change x, c and the patterns as
 * stated beside ACOPF_CARTESIAN and ACOPF_SLACK_* below.  It computes, in
 * FP64:
 *   f       quadratic generator cost on MW:  sum_k c2 (B Pg)^2 + c1 B Pg + c0
 *   grad_f  dense, length n (zeros outside the Pg block)
 *   c       constraints [g^P (nb); g^Q (nb); h^f (nl); h^t (nl)]
 *           g = bus injection - generation + load; h = squared apparent flow
 *   J       values of dc/dx on the fixed CSR pattern of acopf_pattern
 *   H       values of the lower triangle of sigma grad^2 f + sum lambda_r grad^2 c_r
 *   u       vector-Jacobian product  w_f grad f + J' w_c
 *   H d, J d  Hessian- and Jacobian-vector products, neither matrix formed
 * for one net, for a batch of nets in one launch, and for coupling rows that
 * join instances of a batch.
 * Variables x = [theta (nb); v (nb); Pg (ng); Qg (ng)], n = 2 nb + 2 ng;
 * constraints and multipliers in the order of c, m = 2 nb + 2 nl.
 * Branch model: pi model, series admittance 1/(r + j x), charging b/2 at both
 * ends, ideal transformer tap*exp(j shift) on the from side.  Per unit on
 * base_mva; angles in radians.
 *
 * Pattern rule (structural, explicit zeros kept, parallel branches share one
 * slot, columns strictly ascending in each row):
 *   J row g^P_i: theta_j, v_j for j in {i} u N(i), then Pg_k of gens at bus i
 *   J row g^Q_i: the same with Qg
 *   J rows h^f_l, h^t_l: theta_a, theta_b, v_a, v_b with a < b its endpoints
 *   H row theta_i: theta_j for j <= i in {i} u N(i)
 *   H row v_i: theta_j for j in {i} u N(i), then v_j for j <= i
 *   H row Pg_k: Pg_k;  H rows Qg_k: empty.
 *
 * Conventions for every call:
 *   - returns 0 (ACOPF_OK) or a negative ACOPF_E* code; acopf_last_error()
 *     returns a thread-local message for the last failure on this thread;
 *   - no C++ exception crosses the ABI;
 *   - "device" pointers are hipMalloc'd memory of the device the handle was
 *     created on (e.g. torch tensor data pointers); "host" pointers are
 *     ordinary CPU memory;
 *   - evaluation calls are asynchronous: they enqueue work on `stream` and
 *     return; results are valid once the stream is synchronised;
 *   - NaN or Inf in x or the multipliers is not checked; it propagates;
 *   - a handle may be used by one stream at a time (evaluations keep a small
 *     per-handle scratch for the deterministic reduction of f).
 * All results are deterministic: repeated calls, and the same instance
 * evaluated alone or inside any batch, give bitwise identical values.
 *
 * The header is plain C (C11 or C++); a caller compiled without hipcc
 * defines __HIP_PLATFORM_AMD__, as HIP's own headers require, adds
 * /opt/rocm/include to the include path and links libacopf.so.
 */
#ifndef ACOPF_ABI_H_
#define ACOPF_ABI_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ACOPF_OK = 0,
  ACOPF_EINVAL = -1,  /* bad argument, size or network data                */
  ACOPF_ENOMEM = -2,  /* device or host allocation failed                   */
  ACOPF_EHIP = -3,    /* HIP runtime error (message carries the HIP string) */
  ACOPF_EBUDGET = -4, /* request exceeds a memory budget                    */
  ACOPF_ESTATE = -5   /* handle in the wrong state (e.g. still referenced)   */
};

/* `what` bits for the fused and batched evaluations. */
enum {
  ACOPF_F = 1u,      /* objective value           */
  ACOPF_GRADF = 2u,  /* objective gradient (n)    */
  ACOPF_C = 4u,      /* constraint values (m)     */
  ACOPF_J = 8u,      /* Jacobian values           */
  ACOPF_H = 16u,     /* Lagrangian Hessian values */
  ACOPF_ALL = 31u
};

/* Thread-local description of the last error on this thread ("" if none). */
const char* acopf_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int acopf_version(void);

typedef struct acopf_net_s* acopf_net;
typedef struct acopf_batch_s* acopf_batch;

/* Network description.  HOST pointers, read during acopf_net_create and not
 * kept; the caller keeps ownership.  Bus ids are 0-based.  Validation:
 * nbus >= 1, nbranch >= 0, ngen >= 0, base_mva > 0, endpoints in range and
 * distinct, not both r and x zero, tap > 0, generator buses in range,
 * every value finite.  Parallel branches are allowed.  br_rate is not used
 * by the evaluation; it sets the flow rows' upper bounds (acopf_flow_limits,
 * the h+ of the OPFLOW section's inequality h- <= h(x) <= h+). */
typedef struct {
  int32_t nbus, nbranch, ngen;
  double base_mva;                  /* the cost is on MW = base_mva * Pg   */
  const int32_t* br_from;           /* [nbranch]                           */
  const int32_t* br_to;             /* [nbranch]                           */
  const double* br_r;               /* [nbranch] series resistance, pu     */
  const double* br_x;               /* [nbranch] series reactance, pu      */
  const double* br_b;               /* [nbranch] total charging, pu        */
  const double* br_tap;             /* [nbranch] tap ratio (1 for lines)   */
  const double* br_shift;           /* [nbranch] phase shift, rad          */
  const double* br_rate;            /* [nbranch] apparent-power limit, pu;
                                       <= 0: unlimited                     */
  const double* bus_pd;             /* [nbus] active load, pu              */
  const double* bus_qd;             /* [nbus] reactive load, pu            */
  const double* bus_gs;             /* [nbus] shunt conductance at v = 1   */
  const double* bus_bs;             /* [nbus] shunt susceptance at v = 1   */
  const int32_t* gen_bus;           /* [ngen]                              */
  const double* gen_c2;             /* [ngen] $/MW^2h                      */
  const double* gen_c1;             /* [ngen] $/MWh                        */
  const double* gen_c0;             /* [ngen] $/h                          */
} acopf_net_desc;

typedef struct {
  int64_t n;         /* 2 nbus + 2 ngen (+ nbus per slack block)           */
  int64_t m;         /* 2 nbus + 2 (live branches) (+ nbus, cartesian)     */
  int64_t m_eq;      /* equality rows g = 0, the first 2 nbus rows of c    */
  int64_t nnz_jac;   /* Jacobian pattern entries                           */
  int64_t nnz_hess;  /* lower-Hessian pattern entries                      */
  int32_t nbus, nbranch, ngen;
  int32_t outage;    /* removed branch of an N-1 net, -1 for a base net    */
} acopf_dims;

/* Create a network on the current HIP device: validates `desc`, derives the
 * branch admittances, the bus adjacency and the CSR patterns on the host and
 * uploads them.  Errors: EINVAL (validation, with the offending index in the
 * message, or a bus whose rows exceed the per-tile capacity), ENOMEM, EHIP. */
int acopf_net_create(const acopf_net_desc* desc, acopf_net* out);

/* N-1 child of a base net (paper: SCOPFLOW section, contingency cases of the
 * security-constrained problem): branch `branch` of `base` is removed
 * entirely.  Its two flow rows disappear (m drops by 2; later flow rows shift
 * down by one) and its Jacobian/Hessian slots vanish unless a parallel branch
 * still joins the same buses.  x keeps the base layout.  The child shares the
 * base's device network data (it adds only a few bytes of scratch for the
 * reduction of f); `base` cannot be destroyed while children exist (ESTATE).
 * Errors: EINVAL, ESTATE, ENOMEM. */
int acopf_net_create_outage(acopf_net base, int32_t branch, acopf_net* out);

/* Destroy a net.  ESTATE if a child net or a batch still references it. */
int acopf_net_destroy(acopf_net net);

int acopf_dims_get(acopf_net net, acopf_dims* out);

/* CSR patterns of J (m rows) and of the lower Hessian (n rows), as defined
 * above, copied into caller-owned HOST arrays of sizes m+1, nnz_jac, n+1,
 * nnz_hess.  Any pointer may be NULL to skip that array. */
int acopf_pattern(acopf_net net, int32_t* jac_rowptr, int32_t* jac_col,
                  int32_t* hess_rowptr, int32_t* hess_col);

/* Upper bounds h+ of the flow rows (paper: OPFLOW section, h- <= h(x) <= h+
 * with h the squared apparent flows): hmax[r] = rate^2 for flow row r, in the
 * order of c (from ends of the live branches, then their to ends), +inf for a
 * branch whose rate is <= 0; the lower bounds are 0.  hmax: caller-owned HOST
 * array of 2 (live branches) entries.  Errors: EINVAL. */
int acopf_flow_limits(acopf_net net, double* hmax);

/* acopf_flow_limits for a description (no device needed); `outage` = -1 for
 * the base network, else the branch to remove. */
int acopf_flow_limits_host(const acopf_net_desc* desc, int32_t outage, double* hmax);

/* Host-only form of acopf_pattern for a description (no device needed):
 * fills *dims (may be NULL) and, where non-NULL, the four arrays.
 * `outage` = -1 for the base network, else the branch to remove. */
int acopf_pattern_host(const acopf_net_desc* desc, int32_t outage, acopf_dims* dims,
                       int32_t* jac_rowptr, int32_t* jac_col,
                       int32_t* hess_rowptr, int32_t* hess_col);

/* Representation of the network equations (paper: OPFLOW section, the
 * formulations it lists beside the polar power balance).
 *
 * ACOPF_POLAR (what acopf_net_create builds): everything above.
 *
 * ACOPF_CARTESIAN, the power-balance-cartesian form: bus voltages are
 * V_i = e_i + j f_i, so x = [e (nb); f (nb); Pg (ng); Qg (ng)] and, with
 * A = e_f e_t + f_f f_t and B = f_f e_t - e_f f_t,
 *   P_f =  g_ff |V_f|^2 + g_ft A + b_ft B,   Q_f = -b_ff |V_f|^2 + g_ft B - b_ft A,
 *   P_t =  g_tt |V_t|^2 + g_tf A - b_tf B,   Q_t = -b_tt |V_t|^2 - g_tf B - b_tf A,
 * with the same admittances as the polar form; the shunt and load terms use
 * |V_i|^2 = e_i^2 + f_i^2.  c gains nb rows after the flow rows,
 *   c = [g^P; g^Q; h^f; h^t; e_i^2 + f_i^2 (nb)],   m = 3 nb + 2 nl,
 * the squared voltage magnitudes that carry the voltage bounds in this form.
 * Pattern: every polar rule with theta -> e and v -> f, then one J row per
 * bus with columns e_i, f_i (nnz_jac grows by 2 nb); the H pattern is
 * unchanged (the magnitude rows add only diagonal entries).  Every entry
 * point below (single net, N-1 child, batch, products) evaluates both forms;
 * an N-1 child keeps its base's form; a batch needs one form throughout, and
 * acopf_batch_draw_iterates serves only the polar one (EINVAL otherwise). */
enum { ACOPF_POLAR = 0, ACOPF_CARTESIAN = 1 };

/* Feasibility slack variables (paper: OPFLOW section, the formulation
 * features beside the standard ACOPF: load loss and power imbalance).  The
 * paper gives no equations; the model evaluated here:
 *   ACOPF_SLACK_IMBALANCE  four variables per bus, dP+ and dP- in the bus's
 *                          active balance row, dQ+ and dQ- in its reactive
 *                          row; "+" supplies power (coefficient -1, as
 *                          generation), "-" absorbs it (+1, as load);
 *   ACOPF_SLACK_LOADLOSS   two per bus, Pl and Ql, the shed part of the
 *                          bus load (coefficient -1: Pd - Pl remains).
 * Each enabled block holds nb variables; the blocks follow Qg in x in the
 * order dP+, dP-, dQ+, dQ-, Pl, Ql, so n = 2 nb + 2 ng + ns nb with
 * ns in {0, 2, 4, 6}.  Each slack s adds c2 (B s)^2 + c1 (B s) to f
 * (B = base_mva; (c2, c1) = (imb_c2, imb_c1) or (loss_c2, loss_c1)).  The
 * bounds (s >= 0, Pl <= Pd) are the solver's.  Patterns: each balance row
 * gains its slack columns after its generator columns, in block order; H
 * gains one diagonal entry per slack column (explicit zeros kept), after
 * the (empty) Qg rows.  Slacks combine with either representation; N-1
 * children inherit them; acopf_batch_draw_iterates refuses nets with them. */
enum { ACOPF_SLACK_IMBALANCE = 1u, ACOPF_SLACK_LOADLOSS = 2u };

/* Options of a net; a zero-initialised struct is the polar model without
 * slacks (what acopf_net_create builds). */
typedef struct {
  int32_t form;            /* ACOPF_POLAR or ACOPF_CARTESIAN                   */
  uint32_t slacks;         /* ACOPF_SLACK_* bits                               */
  double imb_c2, imb_c1;   /* penalty per imbalance variable, $/MW^2h, $/MWh   */
  double loss_c2, loss_c1; /* penalty per load-loss variable                   */
} acopf_net_opts;

/* acopf_net_create with options (NULL: the defaults).  EINVAL for an unknown
 * form or slack bit or a non-finite penalty. */
int acopf_net_create_opts(const acopf_net_desc* desc, const acopf_net_opts* opts,
                          acopf_net* out);

/* acopf_pattern_host with options (NULL: the defaults). */
int acopf_pattern_host_opts(const acopf_net_desc* desc, const acopf_net_opts* opts,
                            int32_t outage, acopf_dims* dims, int32_t* jac_rowptr,
                            int32_t* jac_col, int32_t* hess_rowptr, int32_t* hess_col);

/* acopf_net_create in the representation `form` (EINVAL for another value). */
int acopf_net_create_form(const acopf_net_desc* desc, int32_t form, acopf_net* out);

/* The representation of a net (its base's, for an N-1 child). */
int acopf_net_form(acopf_net net, int32_t* form);

/* acopf_pattern_host in the representation `form`. */
int acopf_pattern_host_form(const acopf_net_desc* desc, int32_t form, int32_t outage,
                            acopf_dims* dims, int32_t* jac_rowptr, int32_t* jac_col,
                            int32_t* hess_rowptr, int32_t* hess_col);

/* f (1 value), grad_f (n) and c (m) at x (n); DEVICE pointers.  Any output
 * may be NULL to skip it (x may not). */
int acopf_eval_f_g(acopf_net net, const double* x, double* f, double* grad_f,
                   double* c, hipStream_t stream);

/* Jacobian values (nnz_jac, pattern order) at x; DEVICE pointers. */
int acopf_eval_jac(acopf_net net, const double* x, double* jac_val, hipStream_t stream);

/* Lower Lagrangian-Hessian values (nnz_hess) of sigma f + lambda'c at x;
 * lambda has m entries in the order of c; DEVICE pointers, sigma by value. */
int acopf_eval_hess(acopf_net net, const double* x, double sigma, const double* lambda,
                    double* hess_val, hipStream_t stream);

/* u = w_f grad f(x) + J(x)' w_c, without forming J; w_c has m entries;
 * u has n.  DEVICE pointers.  With (w_f, w_c) = (sigma, lambda) this is the
 * gradient of the Lagrangian. */
int acopf_vjp(acopf_net net, const double* x, double w_f, const double* w_c, double* u,
              hipStream_t stream);

/* Hessian-vector product of the Lagrangian without forming H:
 * out = (sigma grad^2 f + sum_r lambda_r grad^2 c_r) d, all n entries (the full
 * symmetric H, not only its lower triangle).  DEVICE pointers: x, d, out (n),
 * lambda (m).  Lets Newton-Krylov solvers skip storing H. */
int acopf_hvp(acopf_net net, const double* x, double sigma, const double* lambda,
              const double* d, double* out, hipStream_t stream);

/* Jacobian-vector product without forming J: out = J(x) d (m entries);
 * DEVICE pointers x, d (n), out (m). */
int acopf_jvp(acopf_net net, const double* x, const double* d, double* out, hipStream_t stream);

/* Everything at once in a single launch: the outputs selected by `what`
 * (ACOPF_* bits; the matching pointer must be non-NULL).  lambda is needed
 * only for ACOPF_H. */
int acopf_eval_all(acopf_net net, const double* x, double sigma, const double* lambda,
                   double* f, double* grad_f, double* c, double* jac_val, double* hess_val,
                   unsigned what, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched evaluation (paper: SCOPFLOW and SOPFLOW sections -- many
 * contingency or scenario subproblems, each evaluated independently; the
 * embarrassingly parallel structure).  Instance k uses nets[k]; its data lives
 * in packed DEVICE buffers at the offsets returned by acopf_batch_offsets:
 * x at x_off[k] (length n_k), lambda and c at c_off[k] (m_k), jac_val at
 * j_off[k] (nnz_jac_k), hess_val at h_off[k] (nnz_hess_k), grad_f and u at
 * x_off[k]; sigma, f and w_f are arrays of `count`.  The whole batch runs in
 * one kernel launch (plus a small reduction launch when some instance has
 * several objective chunks), issued as the schedule says: one workgroup per
 * tile or a persistent grid striding over the tile list, launched directly
 * or replayed from a HIP graph captured per buffer set.
 * ---------------------------------------------------------------------- */

/* Tile/schedule configuration chosen by the autotuner (or fixed by hand). */
typedef struct {
  int32_t tile_be;    /* tile class 64, 128, 256 or 512: workgroups of
                         64/128/256/256 threads holding up to 110/220/440/512
                         branch ends and 55/110/220/256 buses per bus tile */
  int32_t grid_mult;  /* workgroups per CU for the persistent grid; 0 = one
                         workgroup per tile (no persistence)               */
  int32_t xcd_group;  /* 1 = map each instance's tiles onto one XCD        */
  int32_t no_graph;   /* 1 = launch directly instead of replaying a graph */
} acopf_sched;

/* Build a batch over `count` nets (they cannot be destroyed while the batch
 * exists): per-instance offsets, the XCD-aware tile list and the device
 * descriptor table.  `sched` may be NULL for the default schedule
 * {256, 0, 1, 0}.  Errors: EINVAL (also when a bus exceeds the tile
 * capacity of the schedule, or the distinct networks' branch work items
 * exceed 2^31 in total), ENOMEM, EHIP. */
int acopf_batch_create(const acopf_net* nets, int32_t count, const acopf_sched* sched,
                       acopf_batch* out);
int acopf_batch_destroy(acopf_batch batch);

/* Offsets into the packed buffers (HOST arrays of count+1 entries each; the
 * last entry is the total length).  Any pointer may be NULL. */
int acopf_batch_offsets(acopf_batch batch, int64_t* x_off, int64_t* c_off, int64_t* j_off,
                        int64_t* h_off);

/* Evaluate the outputs selected by `what` for every instance in one launch
 * (DEVICE pointers; an output not selected may be NULL).  The first call with
 * a given set of buffers captures a HIP graph; later calls with the same
 * buffers replay it. */
int acopf_batch_eval(acopf_batch batch, const double* x, const double* sigma,
                     const double* lambda, double* f, double* grad_f, double* c,
                     double* jac_val, double* hess_val, unsigned what, hipStream_t stream);

/* Batched VJP: u_k = w_f[k] grad f_k + J_k' w_c_k for every instance. */
int acopf_batch_vjp(acopf_batch batch, const double* x, const double* w_f, const double* w_c,
                    double* u, hipStream_t stream);

/* Batched Hessian- and Jacobian-vector products: per instance, out_k =
 * H_k d_k (packed like x; sigma is a DEVICE array of count) and
 * out_k = J_k d_k (packed like c). */
int acopf_batch_hvp(acopf_batch batch, const double* x, const double* sigma,
                    const double* lambda, const double* d, double* out, hipStream_t stream);
int acopf_batch_jvp(acopf_batch batch, const double* x, const double* d, double* out,
                    hipStream_t stream);

/* Per-instance dot products over the packed x layout: out[k] = a_k . v_k,
 * the sum over the n_k entries of instance k (a, v packed like x; out has
 * count entries; DEVICE pointers), added in a fixed order.  With a = grad f
 * it is the directional derivative of each objective, which the second-order
 * adjoint of the batched VJP needs for the weight w_f.  Errors: EINVAL, EHIP. */
int acopf_batch_xdot(acopf_batch batch, const double* a, const double* v, double* out,
                     hipStream_t stream);

/* As acopf_batch_eval, for the instances [first, first + count) only (same
 * packed buffers and offsets; other instances' outputs are not touched).
 * Launched directly, not through a graph: the window changes from call to
 * call, as it does for a continuously batched request stream.  Concurrent
 * calls on one batch must use disjoint windows.  Errors: EINVAL (empty or
 * out-of-range window, null outputs as in acopf_batch_eval), EHIP. */
int acopf_batch_eval_range(acopf_batch batch, int32_t first, int32_t count, const double* x,
                           const double* sigma, const double* lambda, double* f,
                           double* grad_f, double* c, double* jac_val, double* hess_val,
                           unsigned what, hipStream_t stream);

/* acopf_batch_eval for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, outputs and errors as acopf_batch_eval, and
 * bitwise the same results; the call itself allocates nothing (no hipMalloc,
 * hipFree or graph instantiation: the batch is always launched directly).
 * The objective partials of instances with several cost-item chunks (one
 * chunk per 1,024 generators or 2,048 slack variables, at least one per
 * instance) go to a fixed device array of 32,768 doubles (256 KiB) that the
 * library holds on each device it runs on until the process ends; a batch
 * whose chunks exceed that count is refused with EINVAL before anything is
 * launched.  Every call on one device shares that array and nothing in it
 * needs to start at zero, but calls that overlap in time on one device
 * (other streams, other threads) race on it: serialise them. */
int acopf_batch_eval_noalloc(acopf_batch batch, const double* x, const double* sigma,
                             const double* lambda, double* f, double* grad_f, double* c,
                             double* jac_val, double* hess_val, unsigned what,
                             hipStream_t stream);

/* One served window in one call: draws the iterates of the instances
 * [first, first + count) from the request seeds as acopf_batch_draw_iterates
 * does (same stream of numbers), sets their sigma to 1 and evaluates every
 * output as acopf_batch_eval_range with ACOPF_ALL.  seeds: HOST array of
 * count entries, copied into the launch arguments (no device staging, no
 * wait for the host array afterwards); count <= 64.  x, lambda, sigma and the
 * outputs: the batch's packed DEVICE buffers.  The serving loop's fast path
 * for requests that carry only a seed.  Errors: EINVAL (window, count, a
 * cartesian batch or nets with slack variables), EHIP. */
int acopf_batch_serve_window(acopf_batch batch, int32_t first, int32_t count,
                             const uint64_t* seeds, double pmin, double pmax, double qmin,
                             double qmax, double* x, double* lambda, double* sigma, double* f,
                             double* grad_f, double* c, double* jac_val, double* hess_val,
                             hipStream_t stream);

/* Random iterates for the instances [first, first + count), drawn on the
 * device for a served request stream (the request carries only a seed).
 * Counter-based: stream element j of instance k is
 *   u = (splitmix64(seeds[k] + (j + 1) * 0x9E3779B97F4A7C15) >> 11) * 2^-53
 * with the SplitMix64 output function of Steele, Lea and Flood (2014).
 * x: theta = -0.2 + 0.4 u, v = 0.95 + 0.1 u, Pg = pmin + (pmax - pmin) u,
 * Qg = qmin + (qmax - qmin) u, from elements 0 .. n-1 in x order; lambda_r is
 * the Box-Muller normal sqrt(-2 ln(1 - u1)) cos(2 pi u2) of elements
 * n + 2r and n + 2r + 1.  seeds: DEVICE array indexed by instance (the batch's
 * count entries); x and lambda: the packed DEVICE buffers.  Errors: EINVAL, EHIP. */
int acopf_batch_draw_iterates(acopf_batch batch, int32_t first, int32_t count,
                              const uint64_t* seeds, double pmin, double pmax, double qmin,
                              double qmax, double* x, double* lambda, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Coupling rows between instances of a batch (paper: SCOPFLOW, TCOPFLOW and
 * SOPFLOW sections -- the contingency, time and scenario coupling
 * constraints  -delta <= x_a - x_b <= delta  that join subproblems into one
 * block-structured NLP; here on generator real power, the paper's example of
 * such a coupling).  Link l joins instance child[l] to instance parent[l]
 * (a contingency to its base case, a period to the one before it, a
 * scenario to the base).  Its row block holds, for each generator k in
 * order, the row  Pg_k(child) - Pg_k(parent); blocks follow the links'
 * order.  The bounds +-delta belong to the solver; the rows are linear, so
 * they add nothing to H.  With the batch's per-instance blocks, the coupled
 * problem's constraints are [c_0; ...; c_{K-1}; rows] over x = the packed x.
 * ---------------------------------------------------------------------- */

typedef struct acopf_couple_s* acopf_couple;

/* child, parent: HOST arrays of nlinks instance indices of `batch` (which
 * must outlive the coupling).  Errors: EINVAL (index out of range, a link
 * joining an instance to itself, different generator counts), ENOMEM, EHIP. */
int acopf_couple_create(acopf_batch batch, const int32_t* child, const int32_t* parent,
                        int32_t nlinks, acopf_couple* out);
int acopf_couple_destroy(acopf_couple cp);

/* Number of coupling rows and of their Jacobian nonzeros (two per row). */
int acopf_couple_dims(acopf_couple cp, int64_t* rows, int64_t* nnz);

/* CSR pattern of the rows over the batch's packed x (HOST arrays: rowptr of
 * rows + 1 entries, col of nnz entries; columns ascending in each row). */
int acopf_couple_pattern(acopf_couple cp, int64_t* rowptr, int64_t* col);

/* Row values c[r] = x[child column] - x[parent column] and the Jacobian
 * values (+1 / -1 in pattern order).  DEVICE pointers; c or jac_val may be
 * NULL.  Errors: EINVAL, EHIP. */
int acopf_couple_eval(acopf_couple cp, const double* x, double* c, double* jac_val,
                      hipStream_t stream);

/* u += J' w for the coupling rows: w has one entry per row, u is packed
 * like x and keeps what it holds (add the batch's own VJP first).  Each
 * entry of u is updated by one thread, adding its rows in row order.  DEVICE
 * pointers.  Errors: EINVAL, EHIP. */
int acopf_couple_vjp(acopf_couple cp, const double* w, double* u, hipStream_t stream);

/* out = J d for the coupling rows (out: one entry per row; DEVICE). */
int acopf_couple_jvp(acopf_couple cp, const double* d, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* ACOPF_ABI_H_ */
