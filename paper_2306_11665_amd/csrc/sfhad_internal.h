// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/sfhad.h"

namespace sfhad {

constexpr int kMaxN = 16;

// The 1D operator of Eq. (5): nodes, weights and Q = diag(w) D (row-major),
// and the Lagrange basis at the interval ends, lm[k] = l_k(-1),
// lp[k] = l_k(+1) (the facet interpolation of the surface term).
struct Operator1D {
    int n = 0;
    int node_kind = -1;
    double x[kMaxN];
    double w[kMaxN];
    double Q[kMaxN * kMaxN];
    double lm[kMaxN];
    double lp[kMaxN];
};

bool build_operator(int n, int node_kind, Operator1D &op);
bool get_operator(int n, int node_kind, Operator1D &op);

// Thread-local error detail for sf_last_error().
void set_error(const std::string &msg);

// A fully validated volume-term request.
struct VolumeRequest {
    const double *u = nullptr;
    double *out = nullptr;
    int64_t E = 0;
    int n = 0;
    int d = 0;
    int flux = 0;
    int precision = SF_PREC_FP64;
    double gamma = 1.4;
    hipStream_t stream = nullptr;
    Operator1D op;
    // surface term (the Remark after Eq. (5)): facet states and outputs,
    // [v][e][2d faces][n^(d-1)]; mode selects what a launch computes
    const double *uf = nullptr;
    double *yf = nullptr;
    int mode = 0;
    // curvilinear volume term: the 9 metric-term arrays, [m][k][e][node]
    const double *aux = nullptr;
};
enum { kModeVolume = 0, kModeSurface = 1, kModeVolumeSurface = 2 };

// Kernel launchers (volume_kernels.hip, surface_kernels.hip, dense_kernels.hip).  They return
// SF_OK, SF_ERR_UNSUPPORTED for a shape that is not instantiated, or
// SF_ERR_HIP when the launch fails.
int launch_sf_volume(const VolumeRequest &r);
int launch_sf_surface(const VolumeRequest &r);  // kModeSurface or kModeVolumeSurface
int launch_sf_curvilinear(const VolumeRequest &r);
int launch_dense_volume(const VolumeRequest &r);

// ---------------------------------------------------------------------------
// Serving kernel interface (volume_kernels.hip).
// One request of a batch as the serving kernel sees it.
struct ServeDesc {
    const double *u;     // device state, 5 x E x n^3 (Euler, SoA)
    double *out;         // device output, same layout
    int64_t E;           // elements of the mesh
    int64_t blk_begin;   // first global block index of this request
    int32_t n;           // nodes per direction, 2..kServeMaxN
    int32_t prec;        // sf_precision
    int32_t node_kind;   // sf_node_kind
    int32_t nblk;        // blocks of this request
    double gamma;
};
constexpr int kServeMaxN = 8;

// Blocks (workgroups' work units) a request of E elements with n nodes per
// direction takes in precision prec: ceil(E / elements-per-block).
int64_t serve_blocks(int n, int prec, int64_t E);
// Size in doubles of the operator table and its host-side filling.
int serve_optable_doubles();
void serve_fill_optable(double *host);
// The serving kernel of variant v = prec * 7 + (n - 2); its only
// argument is a ServeArgs, passed by value.
constexpr int kServeVariants = 14;
inline int serve_variant(int n, int prec) { return prec * (kServeMaxN - 1) + (n - 2); }
// The requests of one variant's launch: their descriptors travel in the
// kernel arguments when there are at most kServeInline of them (nothing to
// copy before the launch), else in a device array.
constexpr int kServeInline = 32;
struct ServeArgs {
    const ServeDesc *desc;  // device array of ndesc descriptors, or null: inl holds them
    const double *optab;    // operator table (serve_fill_optable)
    int32_t ndesc;          // requests of this launch
    int32_t total;          // blocks of this launch (sum of nblk)
    ServeDesc inl[kServeInline];
};
const void *serve_variant_kernel(int variant);
// Threads per block of that kernel (its lane mapping's block size).
int serve_threads(int variant);

// Number of conserved variables of a flux kind (0 for an unknown kind).
inline int flux_nvar(int flux) {
    switch (flux) {
        case SF_FLUX_BURGERS_EC: return 1;
        case SF_FLUX_PRODUCT: return 1;
        case SF_FLUX_EULER_CHANDRASHEKAR: return 5;
        case SF_FLUX_EULER_CHANDRASHEKAR_PFIX: return 5;
        default: return 0;
    }
}

}  // namespace sfhad
