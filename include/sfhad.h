/*
 * sfhad.h -- C-ABI of the MI355X (gfx950) sum-factorized Hadamard-product
 * library (libsfhad.so).
 *
 * The library evaluates the flux-differencing volume term of an
 * entropy-conserving high-order scheme on a mesh of E independent hexahedral
 * (d = 3) or quadrilateral (d = 2) elements:
 *
 *     y = sum_{m=0}^{d-1} (A_m o F_m) 1 ,    F_m[i][j] = f_m(u_i, u_j),
 *
 * where A_m is the Kronecker product with the dense 1D operator Q = W D in
 * direction m and the diagonal weight matrix W = diag(w) in every other
 * direction (Eq. (5) of Cicchino & Nadarajah, "Scalable Evaluation of
 * Hadamard Products with Tensor Product Basis for Entropy-Stable High-Order
 * Methods").  Because every factor but one is diagonal, only the d n^(d+1)
 * node pairs that share a grid line carry nonzero coefficients (Eq. (3),
 * Theorem 1); sf_hadamard_volume evaluates the two-point flux on exactly
 * those pairs, dense_hadamard_volume on all n^(2d) pairs (Eq. (1), the
 * direct form the paper's Figure 1 compares against).
 *
 * CONVENTIONS (all entry points)
 *  - Pointers are DEVICE pointers unless the name ends in _host.  The caller
 *    owns every buffer it passes; the library never frees caller memory.
 *  - State and output layout (structure of arrays, FP64):
 *        u[v * E * n^d + e * n^d + node],  node = ix + n*iy + n*n*iz
 *    (x fastest, then y, then z: the ordering of Section 2).  v runs over
 *    the conserved variables: 1 for the scalar fluxes, 5 for Euler in the
 *    order (rho, rho*u, rho*v, rho*w, E).  `out` has the same layout.
 *  - Nodes are on [-1, 1]; Q = diag(w) D with D the collocated Lagrange
 *    derivative matrix; no factor 2 is applied to the Hadamard sum.
 *  - Calls are asynchronous on the given HIP stream (the null stream for the
 *    short forms).  Arguments are validated on the host before any HIP call.
 *  - Errors are negative sf_status values; sf_last_error() returns a
 *    thread-local detail string for the last failing call on that thread.
 *  - Non-physical Euler states (rho <= 0 or p <= 0) are outside the domain:
 *    the result is unspecified (NaN/Inf propagate) and nothing is checked on
 *    the device.  Domain of the Euler kernels (tested at its ends):
 *      FP64:        rho and beta = rho/(2p) in about [1e-30, 1e30] (products
 *                   of up to three such means are formed);
 *      FP32-split:  rho and beta in about [1e-10, 1e10] (FP32 products of up
 *                   to three means);
 *    any ratio of rho or beta between the nodes of one element: the per-node
 *    logarithms are taken against the element's first node, and the FP64
 *    logarithmic mean's relative error grows as
 *    eps (|ln(a/a_0)| + |ln(b/a_0)| + 2) / |ln a - ln b| (a_0 the first
 *    node's value), below about 3e-12 per pair for in-element ratios up to
 *    1e6 (measured: within 1e-12 normwise per element up to 1e6).
 *  - Thread safety: the operator cache is mutex-protected; calls on distinct
 *    streams are independent.
 */
#ifndef SFHAD_H
#define SFHAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SF_OK = 0,
    SF_ERR_ARG = -1,          /* null pointer, negative size, aliasing, bad enum */
    SF_ERR_UNSUPPORTED = -2,  /* valid request outside the built shapes (n, d, flux, precision) */
    SF_ERR_HIP = -3,          /* a HIP runtime call failed; detail in sf_last_error() */
    SF_ERR_NOMEM = -4,        /* a device or host allocation failed */
    SF_ERR_BUDGET = -5,       /* serving: the request can never fit the HBM budget */
    SF_ERR_BUSY = -6,         /* serving: no free slot / budget right now (retry later) */
    SF_ERR_NOT_FOUND = -7     /* serving: unknown mesh or ticket */
} sf_status;

typedef enum {
    SF_FLUX_BURGERS_EC = 0,           /* f(a,b) = (a^2 + ab + b^2)/6, 1 variable */
    SF_FLUX_EULER_CHANDRASHEKAR = 1,  /* Chandrashekar's EC/KEP flux, 5 variables, d = 3 */
    SF_FLUX_PRODUCT = 2,              /* f(a,b) = a b (C_ij = c_i c_j of the Results section) */
    SF_FLUX_EULER_CHANDRASHEKAR_PFIX = 3
    /* Chandrashekar's flux with Ranocha's pressure fix (the flux of the
     * Results section's Taylor-Green runs, cited there, not printed): the
     * momentum flux takes the arithmetic pressure mean {{p}}, and the energy
     * flux the entropy-conservative completion, whose pressure work is
     * (p_L v_R + p_R v_L)/2.  5 variables, d = 3, FP64: the volume term, the
     * dense path, the surface term and the curvilinear volume term (not the
     * FP32-split form or the serving loop). */
} sf_flux_kind;

typedef enum {
    SF_NODES_GAUSS_LEGENDRE = 0,
    SF_NODES_GAUSS_LOBATTO = 1
} sf_node_kind;

typedef enum {
    SF_PREC_FP64 = 0,        /* FP64 throughout */
    SF_PREC_FP32_SPLIT = 1   /* FP32 flux and line sums; FP64 near-equal log-means and direction sum */
} sf_precision;

/* Supported shapes:
 *   d in {2, 3};  scalar fluxes: 2 <= n <= 16;  Euler: d = 3, 2 <= n <= 13;
 *   dense_hadamard_volume additionally needs n^d <= 4096 and SF_PREC_FP64;
 *   SF_PREC_FP32_SPLIT is built for the Euler flux only. */
#define SF_MIN_N 2
#define SF_MAX_N 16
#define SF_MAX_N_EULER 13
#define SF_MAX_N_CURV 10  /* curvilinear Euler term: the staged element must fit in LDS */

/* Optional arguments of the _ex entry points.  Initialise with
 * sf_opts_init() and override fields as needed. */
typedef struct sf_opts {
    int node_kind;              /* sf_node_kind, default SF_NODES_GAUSS_LEGENDRE */
    int precision;              /* sf_precision, default SF_PREC_FP64 */
    double gamma;               /* ratio of specific heats, default 1.4 (Euler only) */
    void *stream;               /* hipStream_t to launch on, default null stream */
    const double *op_1d_host;   /* optional n x n row-major override of Q (host, copied) */
    const double *w_1d_host;    /* optional n override of w (host, copied); both or neither */
} sf_opts;

/* Fill *opts with the defaults listed above.  Returns SF_ERR_ARG on NULL. */
int sf_opts_init(sf_opts *opts);

/* Sum-factorized volume term (Eq. (3) with the coefficients of Eq. (5);
 * Algorithms 1-2 become index arithmetic inside the kernel).
 *   u_nodes    device, n_var * E * n^d doubles, read only
 *   elem_count E >= 0 (E = 0 is a successful no-op)
 *   n          nodes per direction (polynomial degree + 1)
 *   d          dimension, 2 or 3
 *   flux_kind  sf_flux_kind
 *   out        device, n_var * E * n^d doubles, fully overwritten; must not
 *              overlap u_nodes
 * Gauss-Legendre nodes, gamma = 1.4, FP64, null stream. */
int sf_hadamard_volume(const double *u_nodes, int64_t elem_count, int n, int d,
                       int flux_kind, double *out);

/* Dense O(n^(2d)) evaluation of the same term (Eq. (1)/(3) taken literally:
 * every A_m[i][j], zero or not, times f_m(u_i, u_j) for all i, j).  Same
 * arguments and layout as sf_hadamard_volume.  The speed baseline. */
int dense_hadamard_volume(const double *u_nodes, int64_t elem_count, int n, int d,
                          int flux_kind, double *out);

/* As above with options (opts may be NULL for the defaults). */
int sf_hadamard_volume_ex(const double *u_nodes, int64_t elem_count, int n, int d,
                          int flux_kind, double *out, const sf_opts *opts);
int dense_hadamard_volume_ex(const double *u_nodes, int64_t elem_count, int n, int d,
                             int flux_kind, double *out, const sf_opts *opts);

/* ---------------------------------------------------------------------
 * Curvilinear elements (the Results section's warped grids).  The volume
 * term of a curved element uses the metric-averaged two-point flux in
 * reference direction m,
 *     F_m[i][j] = sum_k f_k(u_i, u_j) (Ja^m_k(i) + Ja^m_k(j)) / 2,
 * with f_k the Cartesian Chandrashekar flux in direction k and
 * Ja^m_k = J d xi^m / d x_k the contravariant metric terms at the nodes;
 * y = sum_m (A_m o F_m) 1 as before, in the Cartesian conserved variables.
 *   Ja   device, 9 * E * n^3 doubles, Ja[(3 m + k) * E * n^3 + e * n^3 + node]
 *        (m: reference direction, k: Cartesian component); not written
 *   u, out  as sf_hadamard_volume (d = 3); out must not overlap u or Ja
 * Euler flux only, FP64 only, 2 <= n <= SF_MAX_N_CURV (SF_ERR_UNSUPPORTED
 * otherwise); opts as for the volume term.  With Ja^m_k = delta_mk it equals
 * sf_hadamard_volume. */
int sf_hadamard_volume_curvilinear(const double *u_nodes, const double *metric, int64_t elem_count, int n,
                                   int flux_kind, double *out, const sf_opts *opts);

/* ---------------------------------------------------------------------
 * Surface term (the Remark after Eq. (5): the same Hadamard product with
 * alpha = 0 on the facet cubature nodes).  Face f = 2m + s of an element is
 * the facet xi_m = -1 (s = 0) or +1 (s = 1); its n^(d-1) cubature nodes are
 * the tensor product of the nodes in the other directions, index t with the
 * remaining directions in increasing order, first fastest (for d = 3:
 * m = 0: t = iy + n iz; m = 1: t = ix + n iz; m = 2: t = ix + n iy).  The
 * facet operator is the quadrature-weighted interpolation to the facet,
 *     B_f = l_s^T in direction m, W = diag(w) in the others
 * (l_s[k] = l_k(-1) or l_k(+1), the Lagrange basis of the nodes at the
 * interval end), so with C_f[t][v] = f_m(u_face[t], u_vol[v]):
 *     y_face_f = (B_f o C_f) 1        y_vol = sum_f (B_f o C_f)^T 1.
 * Only the n volume nodes on the line through a facet node have a nonzero
 * coefficient: 2 d n^d flux evaluations per element.
 *   u_vol, y_vol   device, nvar * E * n^d doubles, the volume layout
 *   u_face, y_face device, nvar * E * 2d * n^(d-1) doubles,
 *                  [v][e][f][t]; the facet states (a trace, an interface
 *                  state -- any admissible state)
 *   y_vol and y_face are fully overwritten and must not overlap each other
 *   or an input (SF_ERR_ARG).  opts: node_kind, gamma, stream and the w
 *   override as for the volume term (Q is not used; the facet interpolation
 *   always uses node_kind's end values); FP64 only (SF_ERR_UNSUPPORTED for
 *   the FP32-split precision).  Shapes as sf_hadamard_volume. */
int sf_hadamard_surface(const double *u_vol, const double *u_face, int64_t elem_count, int n, int d,
                        int flux_kind, double *y_vol, double *y_face, const sf_opts *opts);

/* The volume and surface terms in one pass: y_vol = sum_m (A_m o F_m) 1 +
 * sum_f (B_f o C_f)^T 1 and y_face as above (arguments as
 * sf_hadamard_surface; y_vol holds the sum of the two terms). */
int sf_hadamard_volume_surface(const double *u_vol, const double *u_face, int64_t elem_count, int n, int d,
                               int flux_kind, double *y_vol, double *y_face, const sf_opts *opts);

/* Entropy-projected facet states of 3D Euler nodal states, the facet input
 * of the surface term in an entropy-stable scheme:
 *     u_face[t] = u( sum_k l_s[k] v(u_k) )
 * over the n nodes of the line through facet node t of face (m, s), with
 * v = dU/du the entropy variables of U = -rho s/(gamma - 1) and u(.) the
 * inverse map (with as many nodes as modes per direction the L2 projection
 * of v is v itself, so this is u(V_f P v(u))).
 *   u_nodes  device, 5 * E * n^3 doubles, the volume layout
 *   u_face   device, 5 * E * 6 * n^2 doubles, [v][e][f][t] as for
 *            sf_hadamard_surface; fully overwritten; must not overlap u_nodes
 * 2 <= n <= 13, FP64; opts: node_kind, gamma, stream (NULL = defaults).
 * States must be physical (rho, p > 0) and so must the interpolated entropy
 * variables (v_4 < 0); nothing is checked on the device. */
int sf_entropy_trace(const double *u_nodes, int64_t elem_count, int n, double *u_face, const sf_opts *opts);

/* Pointwise maps between the conserved variables u = (rho, rho vel, E) and
 * the entropy variables v = dU/du (U = -rho s/(gamma - 1)) of 3D Euler,
 * over `count` states stored as 5 arrays of count doubles (in[k*count + i]):
 * with the basis transformation they compose the entropy projection
 * u(V P v(u)) on any node set (e.g. over-integrated volume nodes).  In place
 * (out == in) is allowed; asynchronous on `stream` (NULL: null stream);
 * states must be physical (rho, p > 0; v_4 < 0). */
int sf_entropy_variables(const double *u, int64_t count, double *v, double gamma, void *stream);
int sf_conserved_variables(const double *v, int64_t count, double *u, double gamma, void *stream);

/* The Lagrange basis of the n nodes at the interval ends (host, FP64):
 * lm[k] = l_k(-1), lp[k] = l_k(+1); either may be NULL.  No GPU needed. */
int sf_surface_operator_1d(int n, int node_kind, double *lm_host, double *lp_host);

/* The 1D operator the kernels use (FP64, on [-1, 1]): nodes x, weights w and
 * Q = diag(w) D, row-major n x n (Eq. (5)).  Host buffers of n, n and n*n
 * doubles; any of them may be NULL.  No GPU needed. */
int sf_operator_1d(int n, int node_kind, double *x_host, double *w_host, double *Q_host);

/* ---------------------------------------------------------------------
 * Basis transformation (Eq. (6) and the proof of Theorem 1): a modal
 * polynomial basis chi evaluated on the nodes, and its projection Pi with
 * Pi chi = I, applied direction by direction (sum factorization), turns
 * modal coefficients into the nodal values the volume term takes, and back.
 * --------------------------------------------------------------------- */

/* The 1D modal basis: orthonormal Legendre polynomials on [-1, 1],
 * V[q*n + k] = sqrt((2k+1)/2) P_k(x_q) on the n nodes of node_kind, and its
 * projection P = V^{-1} (P V = I).  Host buffers of n*n doubles, row-major;
 * either may be NULL.  No GPU needed.  SF_ERR_ARG for n < 1 or an unknown
 * node kind, SF_ERR_UNSUPPORTED for n outside [2, 16]. */
int sf_basis_1d(int n, int node_kind, double *V_host, double *P_host);

/* out_e = (M (x) ... (x) M) in_e (d factors, the factor of direction m acting
 * on the index along m) for every element e and variable: with M = V the
 * modal coefficients u_hat become nodal values, with M = P the reverse.
 *   in, out   device, nvar * E * n^d doubles, layout [v][e][node] with
 *             node = ix + n iy + n^2 iz (the modal index is ordered the
 *             same way: kx + n ky + n^2 kz).  out may equal in (in place);
 *             any other overlap is SF_ERR_ARG.  out is fully overwritten.
 *   E >= 0 (0 is a no-op), 2 <= n <= 16, d in {2, 3}, nvar >= 1
 *   M_host    host, n*n doubles, row-major, finite; copied before return
 *   stream    a hipStream_t, NULL for the null stream; asynchronous.
 * FP64 throughout (the passes run on the FP64 matrix cores).  Errors as for
 * sf_hadamard_volume, all detected before any HIP call except SF_ERR_HIP. */
int sf_tensor_apply(const double *in, int64_t elem_count, int n, int d, int nvar,
                    const double *M_host, double *out, void *stream);

/* The same with a rectangular 1D matrix: M_host is n_out x n_in (row-major),
 * e.g. n modes to m quadrature nodes (over-integration) or the projection
 * back; in has n_in^d and out n_out^d doubles per (variable, element) slab,
 * layouts as above.  2 <= n_in, n_out <= 16; in place only when
 * n_in == n_out.  sf_tensor_apply is the n_in == n_out case. */
int sf_tensor_apply_rect(const double *in, int64_t elem_count, int n_in, int n_out, int d, int nvar,
                         const double *M_host, double *out, void *stream);

/* Pointwise maps of 3D Euler states (as sf_entropy_variables and
 * sf_conserved_variables below). */
typedef enum {
    SF_MAP_NONE = 0,
    SF_MAP_ENTROPY_VARIABLES = 1,   /* conserved u -> entropy variables v(u) */
    SF_MAP_CONSERVED_VARIABLES = 2  /* entropy variables v -> conserved u(v) */
} sf_post_map;

/* sf_tensor_apply_rect followed by a pointwise map of every output node, in
 * one pass: out = map((M (x) M (x) M) in) for the 5 variables of each of the
 * elem_count elements (d = 3, nvar = 5 implied; layouts as above).  The
 * steps of the uncollocated modal path that end on the quadrature nodes of
 * the over-integration (the proof of Theorem 1): u_q = V u_hat with v(u_q)
 * (n -> n + 2), and the entropy projection u(V P v) with the map back,
 * either as V applied to P v (n -> n + 2) or as the projection V P applied
 * on the quadrature nodes (m -> m).  The map is the same code as the
 * separate map calls: for n_out = n_in + 2 the result is that of
 * sf_tensor_apply_rect then sf_entropy_variables (or sf_conserved_variables)
 * bit for bit, without writing and re-reading the intermediate array.
 *   map       SF_MAP_ENTROPY_VARIABLES or SF_MAP_CONSERVED_VARIABLES
 *   n_out     n_in + 2 with 3 <= n_in <= 8, or n_in with 3 <= n_in <= 10
 *             (else SF_ERR_UNSUPPORTED)
 *   gamma     > 1 (the ratio of specific heats of the map)
 *   out       must not overlap in.
 * States must be physical (rho > 0, p > 0 after the interpolation; -v_4 > 0
 * for the map back); otherwise NaN or Inf propagate as in the map calls.
 * Errors as for sf_tensor_apply_rect. */
int sf_tensor_apply_rect_map(const double *in, int64_t elem_count, int n_in, int n_out, int map, double gamma,
                             const double *M_host, double *out, void *stream);

/* n_modes orthonormal Legendre modes on the m_nodes nodes of node_kind:
 * V_host (m_nodes x n_modes) and the L2 projection P_host
 * = (V^T W V)^{-1} V^T W (n_modes x m_nodes), with P V = I; for
 * m_nodes > n_modes the rule integrates the mass matrix exactly and
 * P = V^T W.  2 <= n_modes <= m_nodes <= 16.  Either pointer may be NULL. */
int sf_basis_rect(int n_modes, int m_nodes, int node_kind, double *V_host, double *P_host);

/* Select the HIP device for the calling thread and build the operators for
 * every n up to n_max (optional warm-up; the first call per shape otherwise
 * does it).  Returns SF_ERR_HIP when no device is usable. */
int sf_init(int device, int n_max);

/* Human-readable name of a status code (static storage). */
const char *sf_status_string(int status);

/* Detail of the last failing call on this thread ("" if none). */
const char *sf_last_error(void);

/* Library version string (static storage). */
const char *sf_version(void);

/* Diagnostic: y[i] = ln(1 + x[i]) as the kernels' staging step computes it
 * (the per-node logarithms of rho and beta relative to the element's first
 * node).  x, y: device arrays of n doubles, x[i] > -1 finite; asynchronous on
 * `stream` (a hipStream_t, NULL for the null stream).  For tests. */
int sf_diag_log1p(const double *x, int64_t n, double *y, void *stream);

/* Diagnostics: y[i] = ln x[i] and y[i] = e^x[i] as the entropy-variable maps
 * compute them (sf_entropy_variables, sf_conserved_variables, sf_entropy_trace
 * and the fused maps of sf_tensor_apply_rect_map).  Same arguments and errors
 * as sf_diag_log1p; any x (ln: -inf at 0, NaN below 0; exp: 0 and +inf beyond
 * the double range).  For tests. */
int sf_diag_log(const double *x, int64_t n, double *y, void *stream);
int sf_diag_exp(const double *x, int64_t n, double *y, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of residual-evaluation requests over          */
/* device-resident meshes of mixed n (one GPU).                               */
/* ------------------------------------------------------------------------ */
typedef struct sf_server sf_server;
typedef int64_t sf_mesh;
typedef int64_t sf_ticket;

/* Create a server on the current device.  hbm_budget_bytes bounds the
 * device memory held by request outputs from admission to sf_release (one
 * device allocation of that size, sub-allocated first fit); max_inflight
 * bounds the number of requests holding output memory at once (1..1024).
 * Requests are admitted in submission order (FIFO).  Each scheduler tick
 * launches every admitted request in one batch; up to two batches run at
 * once.  Mesh states are allocated separately (not part of the budget). */
int sf_server_create(size_t hbm_budget_bytes, int max_inflight, sf_server **out);

/* The same scheduler with a simulated device: no HIP call is made, no memory
 * is allocated, and a batch completes us_per_block microseconds per element
 * block after it starts (batches run one after another).  y_dev from sf_wait
 * is NULL.  For capacity planning and host tests. */
int sf_server_create_sim(size_t hbm_budget_bytes, int max_inflight, double us_per_block,
                         sf_server **out);

/* For tests of error handling, simulated servers only (SF_ERR_UNSUPPORTED
 * otherwise): the next `count` batch launches fail as a failed HIP launch
 * would, so their requests complete with SF_ERR_HIP from sf_wait. */
int sf_server_sim_fail_launches(sf_server *srv, int count);

/* Current queue length, requests holding output memory, and budget bytes in
 * use (any pointer may be NULL). */
int sf_server_stats(sf_server *srv, int64_t *queued, int64_t *inflight, int64_t *budget_used);

/* Since creation: batches launched, the most requests packed into one
 * batch, and the most launch slots running at once (2 means a batch started
 * while the previous one was still on the device).  Any pointer may be NULL. */
int sf_server_batch_stats(sf_server *srv, int64_t *batches, int64_t *max_batch_requests,
                          int64_t *max_slots_busy);

/* Register a mesh: the state (layout as above; Euler flux, d = 3,
 * 2 <= n <= 8, gamma = 1.4) is copied to a device buffer the server owns.
 * u_host_or_dev points to host memory or to device memory of this GPU (the
 * runtime tells them apart); the copy completes before the call returns, so
 * the caller may free or reuse it then.  Returns SF_ERR_UNSUPPORTED for
 * other fluxes or n. */
int sf_mesh_register(sf_server *srv, const double *u_host_or_dev, int64_t elem_count, int n,
                     int flux_kind, int node_kind, sf_mesh *out);

/* Submit one residual evaluation of a registered mesh (non-blocking).
 * SF_ERR_BUDGET if its output (5 E n^3 doubles) exceeds the whole budget. */
int sf_submit(sf_server *srv, sf_mesh mesh, int precision, sf_ticket *out);

/* Non-blocking completion check: 1 if done, 0 if not, <0 on error. */
int sf_poll(sf_server *srv, sf_ticket ticket);

/* Block until the ticket completes; *y_dev points to the result (device,
 * owned by the server until sf_release), *latency_s is submit-to-completion
 * time on the host clock.  Either output pointer may be NULL.  If the batch
 * the request was in could not be launched, returns SF_ERR_HIP (detail in
 * sf_last_error) with *y_dev = NULL; the ticket must still be released. */
int sf_wait(sf_server *srv, sf_ticket ticket, const double **y_dev, double *latency_s);

/* Return a completed ticket's output buffer to the budget. */
int sf_release(sf_server *srv, sf_ticket ticket);

/* Free a mesh; SF_ERR_BUSY while requests on it are not released. */
int sf_mesh_unregister(sf_server *srv, sf_mesh mesh);
/* Stop the scheduler, wait for running batches, free everything. */
int sf_server_destroy(sf_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SFHAD_H */
