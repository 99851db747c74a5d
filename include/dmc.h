/* dmc.h -- C ABI of the MI355X diagrammatic Monte Carlo hot path.
 *
 * What the library computes (paper: "An AI-powered Technology Stack for Solving Many-Electron
 * Field Theory", arXiv:2403.18840):
 *   Sigma^(n)(k, i w_0) = int dV sum_t W_t^(n)(V) e^{i w_0 tau_out}      (eq. sigma_integration)
 * for the 3D uniform electron gas (eq. ueg_action) with the Yukawa interaction of
 * eq. interaction_ct, at the lowest fermionic Matsubara frequency w_0 = pi / beta, estimated by
 * importance sampling (eq. nf_mcmc_estimator_qft_final_revised with alpha = 1) under a VEGAS map
 * (Sec. IV) or a learned flow (eq. NFtransform, eq. coupling_layer).  Units: k_F = E_F = 1,
 * eps_k = k^2 - mu, V(q) = 8 pi gamma / (q^2 + lambda), gamma = alpha r_s.
 *
 * Conventions for every call:
 *  - Every call returns dmc_status; DMC_OK is 0.  On error nothing is enqueued and no handle is
 *    changed; dmc_last_error() returns a thread-local message for the last failing call.
 *  - Handles are library-owned (create / destroy pairs).  They are not thread-safe; distinct
 *    handles are independent.
 *  - Pointers documented "device" are caller-owned device memory of the current HIP device;
 *    pointers documented "host" are caller-owned host memory read during the call only.
 *  - Device work is enqueued on `stream` (a hipStream_t passed as void*; NULL = default stream).
 *    Only dmc_estimate, dmc_sampler_refine and the *_read calls synchronise that stream.
 *  - Sample layout is structure-of-arrays: x[d * ld + i] is coordinate d of sample i, with
 *    ld >= n.  For order n the dimension is D = 4n - 1: loop momenta q_0..q_{n-1} as Cartesian
 *    triples (coordinates 0..3n-1), then the times tau_1..tau_{n-1} of interaction lines
 *    1..n-1 (line 0 sits at tau = 0).  External momenta point along z.
 */
#ifndef DMC_H
#define DMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMC_OK = 0,
    DMC_E_INVALID = -1, /* bad argument: null pointer, size out of range, inconsistent instances */
    DMC_E_NOMEM = -2,   /* a host or device allocation failed */
    DMC_E_DEVICE = -3,  /* a HIP runtime call failed; the HIP error string is in dmc_last_error */
    DMC_E_COMPILE = -4, /* run-time compilation of a graph kernel failed; the log is in dmc_last_error */
    DMC_E_STATE = -5,   /* call out of order (e.g. a second eval_batch before accumulate) */
    DMC_E_NUMERIC = -6  /* estimate: some sample weights were non-finite and were dropped */
} dmc_status;

enum { DMC_MAX_ORDER = 6, DMC_MAX_K = 64, DMC_MAX_GROUPS = 8, DMC_MAX_INSTANCES = 64, DMC_MAX_ROOTS = 64,
       DMC_MAX_TAYLOR = 6 };

/* Derivative roots (deriv_mask bits): d/dmu (chemical potential), d/dlambda (screening),
 * d/dk (external momentum), each the (m, l) = (1, 0), (0, 1) coefficient of
 * eq. sigma_xi_dmu_dlambda or the momentum derivative of eq. deltam_partitions. */
enum { DMC_D_MU = 1, DMC_D_LAMBDA = 2, DMC_D_K = 4 };

typedef struct dmc_graph dmc_graph;
typedef struct dmc_sampler dmc_sampler;
typedef struct dmc_accum dmc_accum;

typedef struct {
    int32_t order;         /* n interaction lines, 1..DMC_MAX_ORDER */
    uint32_t deriv_mask;   /* derivative roots to build; 0 = value only */
    int32_t diagram_index; /* -1 = all diagrams; otherwise only diagram #i of the exported list */
    int32_t part_size;     /* diagrams per straight-line part of the generated kernel (its parts share
                              nothing and keep the register set bounded); 0 chooses by graph size */
    int32_t taylor_order;  /* 0: first-order derivative roots along the masked directions (below);
                              T in 1..DMC_MAX_TAYLOR: Taylor mode (Sec. III.B eq. taylor_node; Sec. VI.A
                              eq. sigma_xi_dmu_dlambda): every d^m/dmu^m d^l/dlambda^l with m + l <= T
                              along the masked directions among mu and lambda, and with DMC_D_K also
                              the k derivative of each (eq. deltam_partitions) */
    int32_t deriv_k;       /* 0: derivative roots at every external momentum; m in 1..DMC_MAX_K: only at the
                              first m external momenta of each evaluation (the effective mass needs them at
                              k_F alone, Sec. VI.A eq. eff_mass_ratio); the other momenta's derivative slots
                              receive zero sums (estimate 0 +- 0) and f_out zeros.  Derivative-only code
                              then runs at those m momenta only. */
    int32_t routing;       /* the integration variables of each diagram (every choice integrates to the same
                              self-energy over unbounded momenta; the ball |q| <= 6 cuts each routing off
                              differently, so estimates agree to the cutoff's tail):
                              DMC_ROUTING_PATH: the canonical labelling, loop momenta on chords next to the
                              external momentum's shortest path (most of each diagram independent of k);
                              DMC_ROUTING_BLOCKS: interaction lines and loop momenta taken from the diagram's
                              building blocks (Sec. II.C: eq. sigma_pq, eq. Dyson, eq. vertex3,
                              eq. parquet_eqns, eq. phi_ph, eq. phi_phbar, eq. phi_pp), so that a block shared
                              by many diagrams is evaluated once; k on the shortest path.  Fewer k-independent
                              operations, more per external momentum (graph_query's op counts tell which is
                              cheaper for a launch).  Any other value: DMC_E_INVALID. */
    int32_t spin_deg;      /* the factor of each closed fermion loop in a diagram's weight (-1)^(n+F) g^F (Sec. II.A,
                              eq. sigma_integration; F closed loops): 2 for the electron gas's spin-1/2 fermions (0
                              also means 2), 1 for spinless fermions; any other value: DMC_E_INVALID.  The
                              observable is always Sigma(k, i w_0) at the lowest fermionic Matsubara frequency. */
    int32_t generation;    /* where the diagram set comes from (the same set, ordered differently): DMC_GENERATE_ENUMERATE,
                              the orderly enumeration of bridgeless permutations; DMC_GENERATE_CONSTRUCT, the bottom-up
                              construction of Sec. II.C (eq. sigma_pq, eq. Dyson, eq. vertex3, eq. parquet_eqns,
                              eq. phi_ph, eq. phi_phbar, eq. phi_pp, with the fully irreducible four-point vertices
                              from an orderly generation), sorted by canonical permutation.  Any other value:
                              DMC_E_INVALID. */
} dmc_graph_spec;

enum { DMC_GENERATE_ENUMERATE = 0, DMC_GENERATE_CONSTRUCT = 1 };

enum { DMC_ROUTING_PATH = 0, DMC_ROUTING_BLOCKS = 1 };

typedef struct {
    int32_t order, dim, n_diagrams, n_root_classes;
    int32_t n_momenta, n_g_leaves, n_v_leaves, n_groups;
    int32_t n_parts, part_size; /* straight-line parts of the generated kernel and their size (0: one part) */
    /* operation counts of the graph per sample: [0] add, [1] mul, [2] fma, [3] transcendental.
     * ops_sample: once per sample (k-independent part, per lambda group already multiplied in at
     * evaluation); ops_k: once per (sample, k) for one lambda group (the algorithmic counts: the
     * graph as one straight-line part); ops_naive: the plain sum of products over diagrams per
     * (sample, k) before hoisting and common-subexpression elimination. */
    int64_t ops_sample[4];
    int64_t ops_k[4];
    int64_t ops_naive[4];
    /* as executed by a kernel in parts (each part evaluates the leaves it uses; k-independent code
     * once per chunk of external momenta is not counted here): ops_*_exec >= ops_* */
    int64_t ops_sample_exec[4];
    int64_t ops_k_exec[4];
    int32_t n_roots;      /* roots per (lambda group, k, Re/Im): the accumulator's n_roots */
    int32_t taylor_order; /* as in the spec */
    /* the part of ops_k (and ops_k_exec) that only forms the derivative roots: with spec.deriv_k = m it runs
     * at m momenta, the rest of ops_k at every momentum */
    int64_t ops_k_deriv[4];
    int64_t ops_k_deriv_exec[4];
    int32_t deriv_k;      /* as in the spec */
    int32_t routing;      /* as in the spec */
    int32_t spin_deg;     /* as in the spec (2 when the spec held 0) */
    int32_t generation;   /* as in the spec */
} dmc_graph_info;

/* One physical instance: all instances in one eval_batch share beta and mu; instances that
 * share lambda are evaluated once and differ only by the factor (gamma / gamma_group)^n. */
typedef struct {
    double beta, mu, lambda, gamma;
} dmc_instance;

const char* dmc_last_error(void);
const char* dmc_version(void);

/* ---- graph (Sec. II: diagrams as a computational graph; Sec. V.A: front end / IR / back end) ----
 * Enumerates all connected, one-particle-irreducible self-energy diagrams of the given order
 * with no zero-momentum interaction line (Hartree tadpoles vanish by q != 0 in eq. ueg_action),
 * weight (-1)^(n+F) 2^F, routes their momenta, builds the leaf-deduplicated graph, hoists the
 * k- and lambda-independent part and removes repeated products.  Host only; the device code is
 * compiled lazily at the first evaluation (hiprtc, for gfx950) and its code object is kept in an
 * on-disk cache keyed by source and compiler: directory $DMC_KERNEL_CACHE (set and empty: no
 * cache), else $XDG_CACHE_HOME/dmc-kernels, else $HOME/.cache/dmc-kernels.  Large graphs are
 * emitted in parts (spec.part_size).  *out is library-owned: free with dmc_graph_destroy. */
dmc_status dmc_compile_graph(const dmc_graph_spec* spec, dmc_graph** out);
dmc_status dmc_graph_query(const dmc_graph* g, dmc_graph_info* out);
/* The derivative each root holds: out[3 r + 0..2] = (m, l, e) for root r of d^m/dmu^m d^l/dlambda^l
 * (d/dk)^e of the self-energy (Sec. VI.A, eq. sigma_xi_dmu_dlambda and eq. deltam_partitions).  First-order
 * mode: the value, then d/dmu, d/dlambda, d/dk as masked.  Taylor mode: e = 0 before e = 1; within each,
 * by m + l ascending, then m descending.  cap: ints available at out (3 n_roots needed, else DMC_E_INVALID). */
dmc_status dmc_graph_root_orders(const dmc_graph* g, int32_t* out, int32_t cap);
/* Text export of the diagram list, one diagram per line:
 *   "<sigma_0> ... <sigma_{2n-1}> | w <weight> | ext <line> | G src dst c_0..c_{n-1} c_k ; ... | V ..."
 * buf may be NULL to query the length; *len receives the byte count without the final NUL. */
dmc_status dmc_graph_export_diagrams(const dmc_graph* g, char* buf, size_t cap, size_t* len);
/* Generated device source for the given number of lambda groups (for inspection). */
dmc_status dmc_graph_source(const dmc_graph* g, int32_t n_groups, char* buf, size_t cap, size_t* len);
void dmc_graph_destroy(dmc_graph* g);

/* ---- accumulator (FP64 running sums; the only FP64 arithmetic on the device) ----
 * Holds, per (lambda group, k, Re/Im, root), sum w and sum w^2 in FP64 plus the sample count
 * and the count of non-finite weights.  n_roots (1..DMC_MAX_ROOTS) = the graph's (dmc_graph_info).
 * One evaluation workgroup keeps four waves' FP64 totals of all n_groups n_k 2 n_roots slots in LDS:
 * dmc_eval_batch returns DMC_E_INVALID when they do not fit (about 1900 slots). */
dmc_status dmc_accum_create(int32_t n_groups, int32_t n_k, int32_t n_roots, dmc_accum** out);
dmc_status dmc_accum_reset(dmc_accum* acc, void* stream);
void dmc_accum_destroy(dmc_accum* acc);

/* ---- sampler (Sec. IV: VEGAS map; Appendix A: flow) ----
 * kind DMC_SAMPLER_UNIFORM: unit-cube uniforms through the physical map;
 * kind DMC_SAMPLER_VEGAS: uniforms through a per-dimension grid of n_bins bins, then the map.
 * Physical map: r = R y, cos(theta) = 2y - 1, phi = 2 pi y per loop, tau_j = beta y; Jacobian
 * prod_i 4 pi R r_i^2 * beta^(n-1) times the grid Jacobian. */
enum { DMC_SAMPLER_UNIFORM = 0, DMC_SAMPLER_VEGAS = 1 };
dmc_status dmc_sampler_create(int32_t kind, int32_t order, int32_t n_bins, double beta, double qmax,
                              dmc_sampler** out);
/* Draw samples first_index .. first_index + n - 1 of the Philox4x32-10 stream `seed`
 * (counter (i mod 2^32, i div 2^32, d div 4, 0), key (seed mod 2^32, seed div 2^32)).
 * x: device float[D][ld]; jac: device float[n]. */
dmc_status dmc_sample(dmc_sampler* s, uint64_t seed, uint64_t first_index, int64_t n, float* x, int64_t ld,
                      float* jac, void* stream);
/* Grid edges, host double[D][n_bins + 1]: read or replace (edges must rise from 0 to 1). */
dmc_status dmc_sampler_get_grid(const dmc_sampler* s, double* edges);
dmc_status dmc_sampler_set_grid(dmc_sampler* s, const double* edges, void* stream);
/* One VEGAS refinement from the histogram gathered by dmc_accumulate since the last refine
 * (smoothing, compression with exponent alpha, equal-weight re-gridding; Lepage 1978).
 * Synchronises `stream`.  Clears the histogram. */
dmc_status dmc_sampler_refine(dmc_sampler* s, double alpha, void* stream);
/* The same refinement on the host, for any histogram (FP64, no device): edges host double[dim][n_bins + 1],
 * hist host double[dim][n_bins] (the per-bin sums of the squared importance), out host double[dim][n_bins + 1]
 * receives the new edges (a dimension whose edges would not rise strictly keeps its old ones).
 * dmc_sampler_refine applies it to the histogram it gathered.  DMC_E_INVALID for null pointers, dim < 1,
 * n_bins < 2 or alpha < 0. */
dmc_status dmc_vegas_refine(int32_t dim, int32_t n_bins, const double* edges, const double* hist, double alpha,
                            double* out);
dmc_status dmc_sampler_read_histogram(dmc_sampler* s, double* hist /* host [D][n_bins] */, void* stream);
void dmc_sampler_destroy(dmc_sampler* s);

/* ---- evaluation (the hot kernel) ----
 * For each sample i < n and each external k_ext[j] (host float[n_k]) evaluates the compiled
 * graph, forms w = f(x_i) J_i for every instance group and Re/Im part, and writes per-block FP64
 * partial sums into `acc` (folded by dmc_accumulate).  Instances: host array of n_inst; all must
 * share beta and mu.
 * f_out (nullable): device float[n_groups][n_roots][n_k][2][n]: the integrand f without J.
 * imp_out (nullable): device float[n]: sum over groups, k, Re/Im and the graph's leading importance roots
 * (dmc_graph_set_importance; the value root alone by default) of |w|, for VEGAS adaptation and flow training. */
dmc_status dmc_eval_batch(dmc_graph* g, const dmc_instance* inst, int32_t n_inst, const float* k_ext, int32_t n_k,
                          const float* x, int64_t ld, const float* jac, int64_t n, dmc_accum* acc, float* f_out,
                          float* imp_out, void* stream);

/* Fold the block partials of the last dmc_eval_batch into the running sums in a fixed order.
 * If sampler is not NULL, also add sum over samples in each (dimension, bin) of imp^2 to the
 * sampler's VEGAS histogram; imp is the imp_out buffer of that eval_batch, and the samples must be
 * the sampler's last dmc_sample call (the bins are recomputed from the Philox counters). */
dmc_status dmc_accumulate(dmc_accum* acc, dmc_sampler* sampler, const float* imp, void* stream);

/* ---- evaluation that allocates nothing ----
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): dmc_eval_batch followed by dmc_accumulate(acc, NULL, NULL, stream) in
 * one call, with the per-block FP64 partial sums and non-finite counts in a static device array of the
 * library (4 MiB, DMC_SCRATCH_BYTES; each GPU the library runs on holds its own copy until the process
 * ends) instead of memory the accumulator allocates on demand.  Same arguments and results as that pair
 * (the block count may be smaller, so FP64 sums can differ in their last bits).  It calls no hipMalloc,
 * hipFree or other allocating routine and compiles nothing: the graph's kernel for this number of lambda
 * groups must already be loaded on the current device (one dmc_eval_batch call with the same graph and
 * groups loads it), else DMC_E_STATE; the accumulator must have no pending evaluation (DMC_E_STATE).
 * DMC_E_INVALID when one block's partial sums (2 x 8 B per accumulator slot, plus 4 B) exceed the
 * scratch, and for the argument errors of dmc_eval_batch.  The scratch keeps the last call's contents;
 * every call overwrites what it reads.  Calls on one GPU share the scratch: calls that overlap on one
 * GPU (from any stream or thread) race, so the caller serialises them. */
#define DMC_SCRATCH_BYTES (4u << 20)
dmc_status dmc_eval_accumulate_noalloc(dmc_graph* g, const dmc_instance* inst, int32_t n_inst, const float* k_ext,
                                       int32_t n_k, const float* x, int64_t ld, const float* jac, int64_t n,
                                       dmc_accum* acc, float* f_out, float* imp_out, void* stream);

/* The roots whose weights make up the importance that dmc_eval_batch writes to imp_out: the first n_roots
 * (1..the graph's roots) in root order; 1 (the value alone) after dmc_compile_graph.  A proposal adapted to
 * the importance concentrates where those roots' integrands are large: the separable VEGAS grid does best on
 * the value alone, a learned flow can follow the derivative roots too.  DMC_E_INVALID outside that range. */
dmc_status dmc_graph_set_importance(dmc_graph* g, int32_t n_roots);

/* Mean and standard error of the mean per instance, root, k and Re/Im:
 * mean, stderr_: host double[n_inst][n_roots][n_k][2].  n_nonfinite: host (nullable).  Uses the
 * instances of the last eval_batch.  Synchronises `stream`.  Returns DMC_E_NUMERIC (with valid
 * finite-sample estimates) when non-finite weights were dropped. */
dmc_status dmc_estimate(dmc_accum* acc, double* mean, double* stderr_, int64_t* n_samples, int64_t* n_nonfinite,
                        void* stream);
/* Raw FP64 sums: host double[n_groups][n_roots][n_k][2][2] as (sum w, sum w^2). */
dmc_status dmc_accum_read(dmc_accum* acc, double* sums, int64_t* n_samples, void* stream);

/* ---- learned proposal: affine-coupling normalizing flow (Appendix A, eq. coupling_layer,
 * eq. NFtransform) ----
 * The flow acts on the VEGAS coordinates u' in (0,1)^D: Philox uniforms u -> z_0 = logit(u) ->
 * n_layers affine couplings z_B <- z_B exp(s) + t, (s_hat, t) = MLP(sigmoid(z_A)) with s = 2 tanh(s_hat) ->
 * u' = sigmoid(z_K) -> the sampler's VEGAS grid -> physical map.  The MLP is in(16) -> 128 -> 128 ->
 * 32 with ReLU; its matmuls run on BF16 MFMA with FP32 accumulation; FP32 master weights.
 * masks: host int8[n_layers][dim], 1 = conditioning (at most 15 per layer), 0 = transformed (at
 * most 16); both sets non-empty.  Parameters: host float[n_layers][22688], per layer
 * W1t[128][16] (column d_A = first-layer bias), W2t[128][128], b2[128], W3t[32][128], b3[32];
 * s_hat_b = output b, t_b = output 16 + b. */
typedef struct dmc_flow dmc_flow;
dmc_status dmc_flow_create(int32_t dim, int32_t n_layers, const int8_t* masks, dmc_flow** out);
/* The paper's flow (Appendix A): coupling layers whose transformed coordinates go through monotonic
 * rational-quadratic splines with 8 bins on [0, 1], parameters from a residual network with two hidden
 * layers of 32 ReLU units (a1 = relu(W1 z_A + b1), a2 = relu(W2 a1 + b2) + a1, theta = W3 a2 + b3), and a
 * uniform base on [0, 1]^dim.  Spline parameters of a transformed coordinate: 8 width logits, 8 height
 * logits, 7 interior derivative logits; widths and heights 1e-3 + (1 - 8e-3) softmax, interior derivatives
 * 1e-3 + softplus, boundary derivatives 1.  Parameters: one FP32 vector, per layer W1 [32][dA], b1 [32],
 * W2 [32][32], b2 [32], W3 [23 dB][32], b3 [23 dB] (row-major; dA, dB: the layer's kept and transformed
 * counts), layers in order.  Created as the identity flow: output layer zero, hidden weights He-normal
 * from a fixed seed (so that every weight receives a gradient).  Every dmc_flow_* call below accepts it; its
 * sampling, density and training run in FP32 on the vector units. */
dmc_status dmc_flow_create_spline(int32_t dim, int32_t n_layers, const int8_t* masks, dmc_flow** out);
dmc_status dmc_flow_param_count(const dmc_flow* f, int64_t* n_params);
dmc_status dmc_flow_set_params(dmc_flow* f, const float* theta, void* stream);  /* also resets Adam state */
dmc_status dmc_flow_get_params(dmc_flow* f, float* theta, void* stream);
/* n samples i = first .. first + n - 1 from the defensive mixture
 *     a_f q_flow + a_g q_grid + a_u q_uniform,   a_f = mix_flow, a_u = mix_uniform, a_g = 1 - a_f - a_u,
 * (in the spirit of the alpha-mixed target of eq. target_distr_nf_mcmc_qft_revised): samples
 * [0, n_u) are uniform points y (the uniform sampler's Philox draw, counters first ..), samples
 * [n_u, n_u + n_g) are the VEGAS sampler's own points (counters first + n_u ..), the rest go through
 * the flow (counters first + n_u + n_g ..), with n_u = round(a_u n), n_g = round(a_g n).  Every sample
 * is weighted by the mixture density at its point (balance-heuristic multiple importance sampling,
 * unbiased): jac = J_phys J_V(u') / (a_f q_flow(u') + a_g + a_u J_V(u')), with u' the point's grid
 * coordinates (u' = G^-1(y) for the uniform share) and J_V the grid's Jacobian there, so every weight
 * is within 1/a_g of the grid sampler's and within 1/a_u of the uniform sampler's.
 * s must be a VEGAS sampler of the flow's dimension.  x: device float[D][ld]; jac: device float[n];
 * u_out (nullable): device float[D][ld], the points u'; lq_out (nullable): device float[n], log q_flow(u').
 * mix_flow in (0, 1], mix_uniform in [0, 1), mix_flow + mix_uniform <= 1.  The library keeps a
 * scratch buffer of 2 (n_u + n_g) (+ D n_u without u_out) floats per flow between calls. */
dmc_status dmc_flow_sample(dmc_flow* f, dmc_sampler* s, uint64_t seed, uint64_t first, int64_t n, float* x,
                           int64_t ld, float* jac, float* u_out, float* lq_out, double mix_flow, double mix_uniform,
                           void* stream);
/* log q(u') by the inverse couplings; u: device float[D][ld]; lq: device float[n]. */
dmc_status dmc_flow_log_density(dmc_flow* f, const float* u, int64_t ld, int64_t n, float* lq, void* stream);
/* Random-walk proposals in the base space of a spline flow T (Sec. IV, the optional base-space moves of
 * NF-MCMC), one per chain state.  u_state (device float[D][ld_u]): the states' grid coordinates u' (as
 * the chains keep them).  Each state's base point z = T^-1(u') moves to z' = z + sigma xi wrapped onto
 * [0, 1)^D, xi standard normals: pair j of coordinates (2j, 2j + 1) of chain i = first + index takes the
 * Philox4x32-10 words w0, w1 of counter (i mod 2^32, i div 2^32, j, 1) and key seed, u_k = ((w_k >> 8) +
 * 1/2) 2^-24, r = sqrt(-2 log u0), xi = (r cos 2 pi u1, r sin 2 pi u1) (Box-Muller).  The proposal u'' =
 * T(z') is mapped like dmc_flow_sample's flow share: x (device float[D][ld]), jac (1/q of the mixture with
 * shares mix_flow, mix_uniform and the rest on the grid, as dmc_flow_sample uses them), u_out (device
 * float[D][ld]: u''), jac_flow (the flow's own weight J_phys J_V J_t / q_T(u'')) and jac_flow_state (the
 * same at each state).  Feed them to dmc_chains_step_walk.  DMC_E_INVALID for an affine flow, sigma not
 * positive and finite, or the shapes of dmc_flow_sample. */
dmc_status dmc_flow_walk(dmc_flow* f, dmc_sampler* s, const float* u_state, int64_t ld_u, int64_t n, double sigma,
                         uint64_t seed, uint64_t first, float* x, int64_t ld, float* jac, float* jac_flow, float* u_out,
                         float* jac_flow_state, double mix_flow, double mix_uniform, void* stream);
/* One step of the weighted forward KL L = -sum_i w_i log q(u'_i) / sum_i w_i over n points:
 * u' = u (device float[D][ld]) or, if u is NULL, the Philox uniforms (seed, first .. first+n-1);
 * w: device float[n] >= 0.  lr > 0 applies one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) to the
 * FP32 masters; grad_out (nullable): device float[n_params] receives dL/dtheta; loss (nullable, host)
 * receives L and synchronises the stream. */
dmc_status dmc_flow_train_step(dmc_flow* f, const float* u, int64_t ld, uint64_t seed, uint64_t first, int64_t n,
                               const float* w, double lr, float* grad_out, double* loss, void* stream);
void dmc_flow_destroy(dmc_flow* f);

/* ---- Markov-chain estimator (Sec. IV, eq. target_distr_nf_mcmc_qft_revised and
 * eq. nf_mcmc_estimator_qft_final_revised) ----
 * n independent chains, one per sample lane, with independent proposals: every step the caller draws
 * n proposals from a sampler (dmc_sample or dmc_flow_sample, jac = 1/q at each proposal) and
 * evaluates them with dmc_eval_batch capturing f_out ([G][R][K][2][ld], ld = the chain count or more).
 * The target is pi = alpha q + (1 - alpha) p, p = |f| summed over root 0's slots (every lambda group,
 * external momentum, Re and Im); a chain moves to its proposal x' with probability
 * min(1, pi(x') q(x) / (pi(x) q(x'))), decided in FP64 as u pi(x) q(x') < pi(x') q(x) with u the 24-bit
 * Philox uniform of key `seed`, counter (chain, step) (first word).  The first step takes every valid
 * proposal; a proposal whose q or pi is not finite and positive is never taken, and a chain without a
 * valid state takes its next valid proposal.  A measured step adds, over the chains, f/pi per slot and
 * q/pi, with their squares, to FP64 sums in a fixed order: I = sum f/pi / sum q/pi.  At alpha = 1 every
 * proposal is taken and the estimate is the plain importance-sampling one.  The sums are kept per chain
 * batch: batch b holds chains [b n / B, (b + 1) n / B) (integer division), so the B batches are
 * independent estimates whose scatter gives the error whatever the chains' autocorrelation time.
 * Handles are library-owned; DMC_E_INVALID for n < 1, n_batches outside [1, min(n,
 * DMC_MAX_CHAIN_BATCHES)] or an observable shape outside the accumulator's limits. */
#define DMC_MAX_CHAIN_BATCHES 4096
typedef struct dmc_chains dmc_chains;
/* dim_u > 0 (at most 4 DMC_MAX_ORDER - 1): each chain also keeps its state's coordinates (dim_u floats,
 * e.g. the grid coordinates u' that dmc_flow_sample writes), for dmc_chains_training_data. */
dmc_status dmc_chains_create(int64_t n, int32_t n_batches, int32_t n_groups, int32_t n_k, int32_t n_roots,
                             int32_t dim_u, dmc_chains** out);
/* One step of every chain: chain c takes proposal (c + offset) mod n (columns of f_prop and u_prop,
 * entries of jac_prop), 0 <= offset < n; u_prop (device float[dim_u][ld_u], ld_u >= n) is required when the
 * chains keep coordinates and ignored otherwise.  Draw offset uniformly and afresh every step: a sampler that lays its
 * proposals out by index (dmc_flow_sample puts each mixture component's share in one index range)
 * then still hands every chain a draw from its full density q, which the acceptance test assumes.
 * measure != 0 accumulates the chains' states after the step. */
dmc_status dmc_chains_step(dmc_chains* c, const float* f_prop, int64_t ld, const float* jac_prop, const float* u_prop,
                           int64_t ld_u, int64_t offset, double alpha, uint64_t seed, int32_t measure, void* stream);
/* One random-walk step in the flow's base space (Sec. IV: the optional base-space proposals of NF-MCMC):
 * chain c's proposal is column c, made by dmc_flow_walk from the chain's own state.  jac_prop (1/q of the
 * sampler's mixture, for the target pi) as in dmc_chains_step; jac_flow_prop and jac_flow_state (device
 * float[n]) are the flow's own weights 1/q_T at the proposals and at the current states.  In base
 * coordinates the target is pi / q_T and the move is symmetric, so the proposal is taken when
 * u pi(x) q_T(x') < pi(x') q_T(x), with the step's uniform u as in dmc_chains_step.  A chain without a
 * valid state, or with a q_T that is not finite and positive on either side, stays.  The chains must keep
 * their coordinates (dim_u = the flow's dimension) and have taken an independence step (else
 * DMC_E_INVALID). */
dmc_status dmc_chains_step_walk(dmc_chains* c, const float* f_prop, int64_t ld, const float* jac_prop,
                                const float* jac_flow_prop, const float* jac_flow_state, const float* u_prop,
                                int64_t ld_u, double alpha, uint64_t seed, int32_t measure, void* stream);
/* sums: host double[n_batches][S + 1][2], S = n_groups n_roots n_k 2 slots in the f_out order, per batch:
 * [b][s][0] = sum f_s/pi, [b][s][1] = sum (f_s/pi)^2; row S: sum q/pi and its squares.  n_measured: chain
 * states added (all batches);
 * n_accepted: proposals taken since the last reset.  Measured steps add to per-block running sums on the
 * device (one launch per step); this call folds them into the totals in a fixed order first, so a step costs
 * no fold.  Synchronises `stream`. */
dmc_status dmc_chains_read(dmc_chains* c, double* sums, int64_t* n_measured, int64_t* n_accepted, void* stream);
/* The chain states as training data for a proposal density (Appendix A: samples that represent |f|,
 * generated by MCMC): u (device float[dim_u][ld], ld >= n) receives the states' coordinates and w
 * (device float[n]) the weights p / pi, p = sum of |f| over root 0's slots (w = 1 at alpha = 0, where the
 * chains sample |f| itself; 0 for a chain without a valid state).  Feed them to dmc_flow_train_step.
 * DMC_E_STATE before the first step. */
dmc_status dmc_chains_training_data(dmc_chains* c, float* u, int64_t ld, float* w, void* stream);
/* The chains' whole independence-sampler loop in the library (Sec. IV: Metropolis–Hastings with independent
 * proposals, eq. target_distr_nf_mcmc_qft_revised), thermal + steps steps with no host round trip: each step
 * draws n proposals from the frozen grid sampler s (dmc_sample) or, with a flow, from its mixture (dmc_flow_sample
 * with mix_flow, mix_uniform), evaluates them (dmc_eval_batch into acc, folded by dmc_accumulate: the
 * importance-sampling estimate of the same proposals, and f, device float[S][n], the chains' observables) and takes
 * one dmc_chains_step.  Step t (from 0 in this call) draws Philox counters first + t n of key seed, uses the
 * acceptance key accept_seed and the rotation offset splitmix64(offset_key, t) mod n; steps t < thermal are not
 * measured, and the sums and acceptance count are reset after them.  x (device float[D][ld], ld >= n), jac
 * (device float[n]), f and u (device float[D][ld], needed with a flow when the chains keep coordinates, ignored
 * otherwise) are the caller's buffers.  DMC_E_INVALID for null pointers, negative counts, alpha outside [0, 1],
 * an accumulator or k list whose shape differs from the chains', or chains that keep coordinates without a flow;
 * errors of the calls it makes are passed on (the chains keep the steps already taken). */
dmc_status dmc_chains_run(dmc_chains* c, dmc_graph* g, const dmc_instance* inst, int32_t n_inst, const float* k_ext,
                          int32_t n_k, dmc_sampler* s, dmc_flow* flow, double mix_flow, double mix_uniform,
                          uint64_t seed, uint64_t first, int64_t thermal, int64_t steps, double alpha,
                          uint64_t accept_seed, uint64_t offset_key, float* x, int64_t ld, float* jac, float* f,
                          float* u, dmc_accum* acc, void* stream);
/* Zero the sums and the accepted count (the chain states are kept). */
dmc_status dmc_chains_reset(dmc_chains* c, void* stream);
void dmc_chains_destroy(dmc_chains* c);

/* ---- estimates across iterations and from Markov chains (host, FP64) ---- */
/* Equal-weight combination of n_iter independent iteration estimates of n_values quantities, the way frozen-grid
 * VEGAS iterations are combined (Sec. IV cites Lepage's VEGAS; equal weights avoid the bias of inverse-variance
 * weights estimated from the same samples): means, errs host double[n_iter][n_values]; mean[v] = the average,
 * err[v] = sqrt(sum_i errs[i][v]^2) / n_iter, chi2_dof[v] = sum_i (means[i][v] - mean[v])^2 / errs[i][v]^2 / (n_iter - 1)
 * (NaN with one iteration or a zero error); chi2_dof near 1 says the iterations agree within their errors.
 * DMC_E_INVALID for null pointers or non-positive sizes. */
dmc_status dmc_combine_iterations(int32_t n_iter, int32_t n_values, const double* means, const double* errs,
                                  double* mean, double* err, double* chi2_dof);
/* The fallback from a learned proposal to the VEGAS grid (Sec. IV: a proposal is judged by the product of its
 * variance and its cost).  From one probe iteration of each proposal with the same sample count: err_flow,
 * err_grid host double[n_values] (the standard errors of the quantities that matter, e.g. every (instance, k,
 * Re/Im) of the value root), t_flow, t_grid the probes' times in any one unit, nonfinite_flow the flow probe's
 * dropped weights.  gain = (sum err_grid^2 t_grid) / (sum err_flow^2 t_flow) (0 if either sum is not finite);
 * use_flow = 1 iff nonfinite_flow == 0 and gain >= min_gain.  DMC_E_INVALID for null pointers, n_values < 1,
 * non-positive or non-finite times or a negative min_gain. */
dmc_status dmc_proposal_select(int32_t n_values, const double* err_flow, const double* err_grid, double t_flow,
                               double t_grid, int64_t nonfinite_flow, double min_gain, int32_t* use_flow,
                               double* gain);
/* The ratio estimator of eq. nf_mcmc_estimator_qft_final_revised from the batch sums of dmc_chains_read (host
 * double[n_batches][S + 1][2], S = n_groups n_roots n_k 2): for every slot, I = (sum_b sum f/pi) / (sum_b sum q/pi),
 * error = the scatter of the batch ratios over sqrt(n_batches); per instance (host dmc_instance[n_inst], grouped by
 * lambda in order of first appearance as in dmc_eval_batch) scaled by (gamma / gamma_group)^order.  mean, err: host
 * double[n_inst][n_roots][n_k][2].  Sums of part of a run (e.g. the difference of two reads) give that part's
 * estimate.  DMC_E_INVALID for null pointers, n_batches < 2 or instances whose lambda count is not n_groups;
 * DMC_E_NUMERIC when no chain weight was measured. */
dmc_status dmc_chains_ratio(int32_t n_batches, int32_t n_groups, int32_t n_roots, int32_t n_k, const double* sums,
                            int32_t order, const dmc_instance* inst, int32_t n_inst, double* mean, double* err);
/* The effective-mass coefficients of one order from its graph's root estimates at k_F (Sec. VI.A,
 * eq. deltam_partitions, eq. deltas_partitions): root_orders host int32[3 n_roots] as dmc_graph_root_orders gives
 * them, est host double[n_roots][2] the (Re, Im) estimates at k_F, w_0 = pi / beta.  For every root (m, l, e = 0):
 * nml = (order, m, l), sigma = Re, b = Im / w_0, and a = (m_e / k_F) Re of the root (m, l, 1) (m_e / k_F = 1/2 with
 * eps_k = k^2; 0 without it).  Outputs host [n_roots] (nml [3 n_roots]); *n_out receives the entries written: the
 * input of dmc_effective_mass.  DMC_E_INVALID for null pointers, order or n_roots < 1, beta <= 0. */
dmc_status dmc_mass_table(int32_t order, const int32_t* root_orders, int32_t n_roots, const double* est, double beta,
                          int32_t* nml, double* sigma, double* a, double* b, int32_t* n_out);

/* ---- checkpoint and resume of an integration ----
 * The state that determines what an integration does next, so that a resumed run computes bit for bit what the
 * uninterrupted one would: the sampler's VEGAS grid and the histogram gathered since its last refinement; the
 * flow's FP32 master weights, Adam moments and step count (its BF16 copies are rebuilt from the masters); the
 * accumulator's FP64 sums, sample and non-finite counts and last instances; and the caller's Philox position
 * (seed and the next sample index: the stream is counter-based, so these two numbers are all of it).  Any handle
 * may be NULL (its section is left out on save, not read on load).  Host buffer; native byte order; synchronises
 * `stream`.  Save: with buf NULL (or cap too small: DMC_E_INVALID) *len receives the size needed.  Load: the
 * handles must have the shapes saved (kind, order, bins, beta, q_max; flow kind, dimension, layers, masks;
 * accumulator shape), else DMC_E_INVALID and no handle changes; DMC_E_STATE while an evaluation waits for
 * dmc_accumulate. */
dmc_status dmc_checkpoint_save(const dmc_sampler* s, const dmc_flow* f, const dmc_accum* acc, uint64_t seed,
                               uint64_t next_index, void* buf, size_t cap, size_t* len, void* stream);
dmc_status dmc_checkpoint_load(dmc_sampler* s, dmc_flow* f, dmc_accum* acc, uint64_t* seed, uint64_t* next_index,
                               const void* buf, size_t len, void* stream);

/* ---- throughput probes (the roofline denominators on the device at hand) ----
 * kind 0: FP32 fused multiply-add (unpacked), 1: the hardware 2^x, 2: the hardware reciprocal; each runs
 * 8 x (compute units) blocks of 256 lanes, every lane 8 independent chains of 16 x `work` operations
 * (work: iterations, 1 .. 2^20).  kind 3: a device-to-device copy of `work` bytes (a multiple of 16, up to
 * 64 GiB; the library allocates and frees both buffers).  After one warm-up launch, *ms receives one
 * launch's time (HIP events on `stream`, which is synchronised) and *ops its operations (kind 3: bytes read
 * plus written).  Not for the hot path: it allocates.  DMC_E_INVALID for an unknown kind or work out of
 * range, DMC_E_NOMEM when an allocation fails. */
dmc_status dmc_probe(int32_t kind, int64_t work, double* ms, double* ops, void* stream);

/* ---- renormalisation post-processing and effective mass (host, FP64) ----
 * Sec. III.B (eq. sigma_xi_dmu, eq. counterterm) and Sec. VI.A (eq. sigma_xi_dmu_dlambda with
 * dlambda = -xi lambda_R, eq. dsigma_depsilon_series, eq. deltam_partitions, eq. deltas_partitions,
 * eq. eff_mass_ratio).  Input: n_coef Fermi-surface coefficients, coefficient c of order
 * (n, m, l) = nml[3c..3c+2] (n >= 1 interaction lines, m mu-derivatives, l lambda-derivatives):
 *   sigma_fs[c] = Re Sigma^(n,m,l)(k_F, i w_0)   (standing in for the zero-frequency value)
 *   a[c] = a^(n,m,l) = (m_e / k_F) d Re Sigma^(n,m,l) / dk at k_F   (m_e / k_F = 1/2 when eps_k = k^2)
 *   b[c] = b^(n,m,l) = Im Sigma^(n,m,l)(k_F, i w_0) / w_0            (w_0 = pi / beta)
 * Each table X becomes X(xi) = sum xi^(n+l) dmu(xi)^m / m! (-lambda_R)^l / l! X^(n,m,l) truncated at xi^N.
 * Counterterms (the pole of the full propagator stays at the Fermi surface): delta_mu^(j) = the xi^j
 * coefficient of Sigma(k_F), j = 1..N.  Outputs, host double[N + 1] each (index = power of xi):
 * delta_mu (delta_mu[0] = 0), a_xi, b_xi, mass = the coefficients of (1 - b(xi)) (1 + a(xi))^-1, and
 * mass_partial[j] = the ratio m_eff/m through order j at xi = 1.  DMC_E_INVALID for N outside 1..32, null pointers,
 * lambda_R < 0 or a coefficient with n < 1 or m, l < 0. */
dmc_status dmc_effective_mass(int32_t N, double lambda_R, int32_t n_coef, const int32_t* nml, const double* sigma_fs,
                              const double* a, const double* b, double* delta_mu, double* a_xi, double* b_xi,
                              double* mass, double* mass_partial);

#ifdef __cplusplus
}
#endif
#endif /* DMC_H */
