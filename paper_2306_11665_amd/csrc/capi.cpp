// The C-ABI entry points: argument validation (all of it on the host, before
// any HIP call), operator lookup, and dispatch to the kernel launchers.
#include <cmath>
#include <cstring>
#include <string>

#include "tensor_internal.h"

namespace sfhad {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

int fail(int status, const char *msg) {
    set_error(msg);
    return status;
}

int64_t ipow(int b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// Shared validation of a volume-term request; fills `r` on success.
int validate(const double *u, int64_t E, int n, int d, int flux, double *out, const sf_opts *opts,
             bool dense, VolumeRequest &r) {
    sf_opts o;
    sf_opts_init(&o);
    if (opts) o = *opts;
    if (E < 0) return fail(SF_ERR_ARG, "elem_count must be >= 0");
    if (n < 1) return fail(SF_ERR_ARG, "n must be >= 1");
    if (d < 1) return fail(SF_ERR_ARG, "d must be >= 1");
    const int nv = flux_nvar(flux);
    if (nv == 0) return fail(SF_ERR_ARG, "unknown flux_kind");
    if (o.node_kind != SF_NODES_GAUSS_LEGENDRE && o.node_kind != SF_NODES_GAUSS_LOBATTO)
        return fail(SF_ERR_ARG, "unknown node_kind");
    if (o.precision != SF_PREC_FP64 && o.precision != SF_PREC_FP32_SPLIT)
        return fail(SF_ERR_ARG, "unknown precision");
    if (!(o.gamma > 1.0) || !std::isfinite(o.gamma)) return fail(SF_ERR_ARG, "gamma must be finite and > 1");
    if ((o.op_1d_host == nullptr) != (o.w_1d_host == nullptr))
        return fail(SF_ERR_ARG, "op_1d_host and w_1d_host must be given together");
    if (d > 3 || d == 1) return fail(SF_ERR_UNSUPPORTED, "d must be 2 or 3");
    if (n < SF_MIN_N || n > SF_MAX_N) return fail(SF_ERR_UNSUPPORTED, "n outside [2, 16]");
    if (flux == SF_FLUX_EULER_CHANDRASHEKAR || flux == SF_FLUX_EULER_CHANDRASHEKAR_PFIX) {
        if (d != 3) return fail(SF_ERR_UNSUPPORTED, "the Euler flux is built for d = 3");
        if (n > SF_MAX_N_EULER) return fail(SF_ERR_UNSUPPORTED, "the Euler flux is built for n <= 13");
    }
    if (o.precision == SF_PREC_FP32_SPLIT && flux != SF_FLUX_EULER_CHANDRASHEKAR)
        return fail(SF_ERR_UNSUPPORTED, "the FP32-split form is built for the (plain) Euler flux only");
    if (dense) {
        if (ipow(n, d) > 4096) return fail(SF_ERR_UNSUPPORTED, "dense path needs n^d <= 4096");
        if (o.precision != SF_PREC_FP64) return fail(SF_ERR_UNSUPPORTED, "dense path is FP64 only");
    }
    const int64_t N = ipow(n, d);
    // every byte count derived from E below (state, facet and metric arrays:
    // at most 16 doubles per node and element) must fit in int64
    if (E > 0 && E > INT64_MAX / (N * 16 * (int64_t)sizeof(double)))
        return fail(SF_ERR_ARG, "elem_count too large");
    r.E = E;
    r.n = n;
    r.d = d;
    r.flux = flux;
    r.precision = o.precision;
    r.gamma = o.gamma;
    r.stream = reinterpret_cast<hipStream_t>(o.stream);
    r.u = u;
    r.out = out;
    if (E == 0) return SF_OK;
    if (!u || !out) return fail(SF_ERR_ARG, "null u_nodes or out");
    const size_t bytes = (size_t)(N * nv * E) * sizeof(double);
    const char *ub = reinterpret_cast<const char *>(u), *ob = reinterpret_cast<const char *>(out);
    if (ub < ob + bytes && ob < ub + bytes) return fail(SF_ERR_ARG, "out overlaps u_nodes");
    if (o.op_1d_host) {
        r.op.n = n;
        r.op.node_kind = o.node_kind;
        for (int i = 0; i < n * n; ++i) r.op.Q[i] = o.op_1d_host[i];
        for (int i = 0; i < n; ++i) {
            r.op.w[i] = o.w_1d_host[i];
            r.op.x[i] = 0.0;
        }
    } else if (!get_operator(n, o.node_kind, r.op)) {
        return fail(SF_ERR_UNSUPPORTED, "operator construction failed");
    }
    return SF_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = reinterpret_cast<const char *>(a), *y = reinterpret_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

// The surface term (mode kModeSurface) or volume + surface (kModeVolumeSurface).
int run_surface(const double *u, const double *uf, int64_t E, int n, int d, int flux, double *yv, double *yf,
                const sf_opts *opts, int mode) {
    VolumeRequest r;
    int st = validate(u, E, n, d, flux, yv, opts, false, r);
    if (st != SF_OK || E == 0) return st;
    if (r.precision != SF_PREC_FP64) return fail(SF_ERR_UNSUPPORTED, "the surface term is built in FP64 only");
    if (!uf || !yf) return fail(SF_ERR_ARG, "null u_face or y_face");
    const int nv = flux_nvar(flux);
    const size_t vbytes = (size_t)(ipow(n, d) * nv * E) * sizeof(double);
    const size_t fbytes = (size_t)(2 * d * ipow(n, d - 1) * nv * E) * sizeof(double);
    if (overlaps(yf, fbytes, uf, fbytes) || overlaps(yf, fbytes, u, vbytes) || overlaps(yf, fbytes, yv, vbytes) ||
        overlaps(yv, vbytes, uf, fbytes))
        return fail(SF_ERR_ARG, "outputs overlap each other or an input");
    // the facet interpolation always uses the node kind's own end values
    Operator1D base;
    if (!get_operator(n, r.op.node_kind, base))
        return fail(SF_ERR_UNSUPPORTED, "operator construction failed");
    for (int i = 0; i < n; ++i) {
        r.op.lm[i] = base.lm[i];
        r.op.lp[i] = base.lp[i];
    }
    r.uf = uf;
    r.yf = yf;
    r.mode = mode;
    return launch_sf_surface(r);
}

int run_curvilinear(const double *u, const double *Ja, int64_t E, int n, int flux, double *out,
                    const sf_opts *opts) {
    VolumeRequest r;
    int st = validate(u, E, n, 3, flux, out, opts, false, r);
    if (st != SF_OK) return st;
    if (flux != SF_FLUX_EULER_CHANDRASHEKAR && flux != SF_FLUX_EULER_CHANDRASHEKAR_PFIX)
        return fail(SF_ERR_UNSUPPORTED, "the curvilinear term is built for the Euler fluxes");
    if (r.precision != SF_PREC_FP64) return fail(SF_ERR_UNSUPPORTED, "the curvilinear term is built in FP64 only");
    if (n > SF_MAX_N_CURV) return fail(SF_ERR_UNSUPPORTED, "the curvilinear term is built for n <= 10");
    if (E == 0) return SF_OK;
    if (!Ja) return fail(SF_ERR_ARG, "null metric terms");
    const size_t vbytes = (size_t)(ipow(n, 3) * 5 * E) * sizeof(double);
    const size_t mbytes = (size_t)(ipow(n, 3) * 9 * E) * sizeof(double);
    if (overlaps(out, vbytes, Ja, mbytes)) return fail(SF_ERR_ARG, "out overlaps the metric terms");
    r.aux = Ja;
    return launch_sf_curvilinear(r);
}

int run(const double *u, int64_t E, int n, int d, int flux, double *out, const sf_opts *opts,
        bool dense) {
    VolumeRequest r;
    int st = validate(u, E, n, d, flux, out, opts, dense, r);
    if (st != SF_OK || E == 0) return st;
    return dense ? launch_dense_volume(r) : launch_sf_volume(r);
}

}  // namespace
}  // namespace sfhad

using namespace sfhad;

extern "C" {

int sf_opts_init(sf_opts *opts) {
    if (!opts) return SF_ERR_ARG;
    opts->node_kind = SF_NODES_GAUSS_LEGENDRE;
    opts->precision = SF_PREC_FP64;
    opts->gamma = 1.4;
    opts->stream = nullptr;
    opts->op_1d_host = nullptr;
    opts->w_1d_host = nullptr;
    return SF_OK;
}

int sf_hadamard_volume(const double *u, int64_t E, int n, int d, int flux, double *out) {
    return run(u, E, n, d, flux, out, nullptr, false);
}

int dense_hadamard_volume(const double *u, int64_t E, int n, int d, int flux, double *out) {
    return run(u, E, n, d, flux, out, nullptr, true);
}

int sf_hadamard_volume_ex(const double *u, int64_t E, int n, int d, int flux, double *out,
                          const sf_opts *opts) {
    return run(u, E, n, d, flux, out, opts, false);
}

int dense_hadamard_volume_ex(const double *u, int64_t E, int n, int d, int flux, double *out,
                             const sf_opts *opts) {
    return run(u, E, n, d, flux, out, opts, true);
}

int sf_hadamard_surface(const double *u, const double *uf, int64_t E, int n, int d, int flux, double *yv,
                        double *yf, const sf_opts *opts) {
    return run_surface(u, uf, E, n, d, flux, yv, yf, opts, kModeSurface);
}

int sf_hadamard_volume_surface(const double *u, const double *uf, int64_t E, int n, int d, int flux, double *yv,
                               double *yf, const sf_opts *opts) {
    return run_surface(u, uf, E, n, d, flux, yv, yf, opts, kModeVolumeSurface);
}

int sf_hadamard_volume_curvilinear(const double *u, const double *Ja, int64_t E, int n, int flux, double *out,
                                   const sf_opts *opts) {
    return run_curvilinear(u, Ja, E, n, flux, out, opts);
}

int sf_entropy_trace(const double *u, int64_t E, int n, double *uf, const sf_opts *opts) {
    sf_opts o;
    sf_opts_init(&o);
    if (opts) o = *opts;
    if (E < 0) return fail(SF_ERR_ARG, "elem_count must be >= 0");
    if (n < 1) return fail(SF_ERR_ARG, "n must be >= 1");
    if (o.node_kind != SF_NODES_GAUSS_LEGENDRE && o.node_kind != SF_NODES_GAUSS_LOBATTO)
        return fail(SF_ERR_ARG, "unknown node_kind");
    if (!(o.gamma > 1.0) || !std::isfinite(o.gamma)) return fail(SF_ERR_ARG, "gamma must be finite and > 1");
    if (o.precision != SF_PREC_FP64) return fail(SF_ERR_UNSUPPORTED, "the entropy trace is built in FP64 only");
    if (n < SF_MIN_N || n > SF_MAX_N_EULER) return fail(SF_ERR_UNSUPPORTED, "the entropy trace is built for 2 <= n <= 13");
    if (E == 0) return SF_OK;
    if (!u || !uf) return fail(SF_ERR_ARG, "null u_nodes or u_face");
    if (E > INT64_MAX / (ipow(n, 3) * 5 * (int64_t)sizeof(double))) return fail(SF_ERR_ARG, "elem_count too large");
    const size_t vbytes = (size_t)(ipow(n, 3) * 5 * E) * sizeof(double);
    const size_t fbytes = (size_t)(6 * ipow(n, 2) * 5 * E) * sizeof(double);
    if (overlaps(u, vbytes, uf, fbytes)) return fail(SF_ERR_ARG, "u_face overlaps u_nodes");
    Operator1D op;
    if (!get_operator(n, o.node_kind, op)) return fail(SF_ERR_UNSUPPORTED, "operator construction failed");
    return launch_entropy_trace(u, uf, E, n, o.gamma, op, reinterpret_cast<hipStream_t>(o.stream));
}

namespace {
int entropy_map(const double *in, int64_t count, double *out, double gamma, void *stream, int dir) {
    if (count < 0) return fail(SF_ERR_ARG, "count must be >= 0");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(SF_ERR_ARG, "gamma must be finite and > 1");
    if (count == 0) return SF_OK;
    if (!in || !out) return fail(SF_ERR_ARG, "null in or out");
    if (count > INT64_MAX / (5 * (int64_t)sizeof(double))) return fail(SF_ERR_ARG, "count too large");
    const size_t bytes = (size_t)count * 5 * sizeof(double);
    if (in != out && overlaps(in, bytes, out, bytes)) return fail(SF_ERR_ARG, "out partially overlaps in");
    return launch_entropy_map(in, out, count, gamma, dir, reinterpret_cast<hipStream_t>(stream));
}
}  // namespace

int sf_entropy_variables(const double *u, int64_t count, double *v, double gamma, void *stream) {
    return entropy_map(u, count, v, gamma, stream, 0);
}

int sf_conserved_variables(const double *v, int64_t count, double *u, double gamma, void *stream) {
    return entropy_map(v, count, u, gamma, stream, 1);
}

int sf_surface_operator_1d(int n, int node_kind, double *lm, double *lp) {
    if (n < 1) return fail(SF_ERR_ARG, "n must be >= 1");
    if (node_kind != SF_NODES_GAUSS_LEGENDRE && node_kind != SF_NODES_GAUSS_LOBATTO)
        return fail(SF_ERR_ARG, "unknown node_kind");
    if (n < SF_MIN_N || n > SF_MAX_N) return fail(SF_ERR_UNSUPPORTED, "n outside [2, 16]");
    Operator1D op;
    if (!get_operator(n, node_kind, op)) return fail(SF_ERR_UNSUPPORTED, "operator construction failed");
    if (lm) std::memcpy(lm, op.lm, sizeof(double) * n);
    if (lp) std::memcpy(lp, op.lp, sizeof(double) * n);
    return SF_OK;
}

int sf_operator_1d(int n, int node_kind, double *x, double *w, double *Q) {
    if (n < 1) return fail(SF_ERR_ARG, "n must be >= 1");
    if (node_kind != SF_NODES_GAUSS_LEGENDRE && node_kind != SF_NODES_GAUSS_LOBATTO)
        return fail(SF_ERR_ARG, "unknown node_kind");
    if (n < SF_MIN_N || n > SF_MAX_N) return fail(SF_ERR_UNSUPPORTED, "n outside [2, 16]");
    Operator1D op;
    if (!get_operator(n, node_kind, op)) return fail(SF_ERR_UNSUPPORTED, "operator construction failed");
    if (x) std::memcpy(x, op.x, sizeof(double) * n);
    if (w) std::memcpy(w, op.w, sizeof(double) * n);
    if (Q) std::memcpy(Q, op.Q, sizeof(double) * n * n);
    return SF_OK;
}

int sf_init(int device, int n_max) {
    int count = 0;
    hipError_t err = hipGetDeviceCount(&count);
    if (err != hipSuccess || count == 0) {
        set_error(std::string("no HIP device: ") + (err != hipSuccess ? hipGetErrorString(err) : "count = 0"));
        return SF_ERR_HIP;
    }
    if (device < 0 || device >= count) return fail(SF_ERR_ARG, "device index out of range");
    err = hipSetDevice(device);
    if (err != hipSuccess) {
        set_error(std::string("hipSetDevice: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    if (n_max > SF_MAX_N) n_max = SF_MAX_N;
    Operator1D op;
    for (int n = SF_MIN_N; n <= n_max; ++n) {
        get_operator(n, SF_NODES_GAUSS_LEGENDRE, op);
        get_operator(n, SF_NODES_GAUSS_LOBATTO, op);
    }
    return SF_OK;
}

int sf_basis_1d(int n, int node_kind, double *V, double *P) {
    if (n < 1) return fail(SF_ERR_ARG, "n must be >= 1");
    if (node_kind != SF_NODES_GAUSS_LEGENDRE && node_kind != SF_NODES_GAUSS_LOBATTO)
        return fail(SF_ERR_ARG, "unknown node_kind");
    if (n < SF_MIN_N || n > SF_MAX_N) return fail(SF_ERR_UNSUPPORTED, "n outside [2, 16]");
    if (!build_basis(n, node_kind, V, P)) return fail(SF_ERR_UNSUPPORTED, "basis construction failed");
    return SF_OK;
}

int sf_tensor_apply_rect(const double *in, int64_t E, int n_in, int n_out, int d, int nvar, const double *M_host,
                         double *out, void *stream) {
    if (E < 0) return fail(SF_ERR_ARG, "elem_count must be >= 0");
    if (n_in < 1 || n_out < 1) return fail(SF_ERR_ARG, "n_in and n_out must be >= 1");
    if (d < 1) return fail(SF_ERR_ARG, "d must be >= 1");
    if (nvar < 1) return fail(SF_ERR_ARG, "nvar must be >= 1");
    if (!M_host) return fail(SF_ERR_ARG, "null M_host");
    if (d > 3 || d == 1) return fail(SF_ERR_UNSUPPORTED, "d must be 2 or 3");
    if (n_in < SF_MIN_N || n_in > SF_MAX_N || n_out < SF_MIN_N || n_out > SF_MAX_N)
        return fail(SF_ERR_UNSUPPORTED, "n_in and n_out must be in [2, 16]");
    const int64_t NI = ipow(n_in, d), NO = ipow(n_out, d);
    const int64_t N = NI > NO ? NI : NO;
    if (E > 0 && E > INT64_MAX / (N * nvar * (int64_t)sizeof(double)))
        return fail(SF_ERR_ARG, "elem_count too large");
    for (int i = 0; i < n_in * n_out; ++i)
        if (!std::isfinite(M_host[i])) return fail(SF_ERR_ARG, "M_host has a non-finite entry");
    if (E == 0) return SF_OK;
    if (!in || !out) return fail(SF_ERR_ARG, "null in or out");
    const size_t ibytes = (size_t)(NI * nvar * E) * sizeof(double), obytes = (size_t)(NO * nvar * E) * sizeof(double);
    if (!(in == out && n_in == n_out) && overlaps(in, ibytes, out, obytes))
        return fail(SF_ERR_ARG, "out overlaps in (in place needs n_in == n_out and out == in)");
    TensorRequest r;
    r.in = in;
    r.out = out;
    r.E = E;
    r.n = n_in;
    r.n_out = n_out;
    r.d = d;
    r.nvar = nvar;
    r.stream = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < n_in * n_out; ++i) r.M[i] = M_host[i];
    return launch_tensor_apply(r);
}

int sf_tensor_apply_rect_map(const double *in, int64_t E, int n_in, int n_out, int map, double gamma,
                             const double *M_host, double *out, void *stream) {
    if (map != SF_MAP_ENTROPY_VARIABLES && map != SF_MAP_CONSERVED_VARIABLES)
        return fail(SF_ERR_ARG, "map must be SF_MAP_ENTROPY_VARIABLES or SF_MAP_CONSERVED_VARIABLES");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(SF_ERR_ARG, "gamma must be finite and > 1");
    if (E < 0) return fail(SF_ERR_ARG, "elem_count must be >= 0");
    if (!M_host) return fail(SF_ERR_ARG, "null M_host");
    const bool up = n_out == n_in + 2 && n_in >= 3 && n_in <= 8, sq = n_out == n_in && n_in >= 3 && n_in <= 10;
    if (!(up || sq))
        return fail(SF_ERR_UNSUPPORTED,
                    "the fused map is built for n_out = n_in + 2 (n_in in [3, 8]) or n_out = n_in (n_in in [3, 10])");
    for (int i = 0; i < n_in * n_out; ++i)
        if (!std::isfinite(M_host[i])) return fail(SF_ERR_ARG, "M_host has a non-finite entry");
    const int64_t NI = ipow(n_in, 3), NO = ipow(n_out, 3);
    if (E > 0 && E > INT64_MAX / (NO * 5 * (int64_t)sizeof(double))) return fail(SF_ERR_ARG, "elem_count too large");
    if (E == 0) return SF_OK;
    if (!in || !out) return fail(SF_ERR_ARG, "null in or out");
    if (overlaps(in, (size_t)(NI * 5 * E) * sizeof(double), out, (size_t)(NO * 5 * E) * sizeof(double)))
        return fail(SF_ERR_ARG, "out overlaps in");
    TensorRequest r;
    r.in = in;
    r.out = out;
    r.E = E;
    r.n = n_in;
    r.n_out = n_out;
    r.d = 3;
    r.nvar = 5;
    r.post_map = map;
    r.gamma = gamma;
    r.stream = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < n_in * n_out; ++i) r.M[i] = M_host[i];
    return launch_tensor_apply(r);
}

int sf_tensor_apply(const double *in, int64_t E, int n, int d, int nvar, const double *M_host, double *out,
                    void *stream) {
    return sf_tensor_apply_rect(in, E, n, n, d, nvar, M_host, out, stream);
}

int sf_basis_rect(int n_modes, int m_nodes, int node_kind, double *V, double *P) {
    if (n_modes < 1 || m_nodes < n_modes) return fail(SF_ERR_ARG, "need 1 <= n_modes <= m_nodes");
    if (node_kind != SF_NODES_GAUSS_LEGENDRE && node_kind != SF_NODES_GAUSS_LOBATTO)
        return fail(SF_ERR_ARG, "unknown node_kind");
    if (n_modes < SF_MIN_N || m_nodes > SF_MAX_N) return fail(SF_ERR_UNSUPPORTED, "sizes outside [2, 16]");
    if (!build_basis_rect(n_modes, m_nodes, node_kind, V, P)) return fail(SF_ERR_UNSUPPORTED, "basis construction failed");
    return SF_OK;
}

const char *sf_status_string(int status) {
    switch (status) {
        case SF_OK: return "SF_OK";
        case SF_ERR_ARG: return "SF_ERR_ARG";
        case SF_ERR_UNSUPPORTED: return "SF_ERR_UNSUPPORTED";
        case SF_ERR_HIP: return "SF_ERR_HIP";
        case SF_ERR_NOMEM: return "SF_ERR_NOMEM";
        case SF_ERR_BUDGET: return "SF_ERR_BUDGET";
        case SF_ERR_BUSY: return "SF_ERR_BUSY";
        case SF_ERR_NOT_FOUND: return "SF_ERR_NOT_FOUND";
        default: return "SF_UNKNOWN_STATUS";
    }
}

const char *sf_last_error(void) { return g_last_error.c_str(); }

const char *sf_version(void) { return "sfhad 0.1.0 (gfx950)"; }

}  // extern "C"
