// Internal declarations of the basis-transformation path (tensor_kernels.hip,
// operators.cpp, capi.cpp).
#pragma once

#include "sfhad_internal.h"

namespace sfhad {

// A validated sf_tensor_apply request: out_e = (M (x) ... (x) M) in_e for
// E elements of nvar variables (input slab v * E + e holds n^d doubles, the
// output slab n_out^d; M is n_out x n, row-major).
struct TensorRequest {
    const double *in = nullptr;
    double *out = nullptr;
    int64_t E = 0;
    int n = 0;      // n_in
    int n_out = 0;  // == n for the square kernels
    int d = 0;
    int nvar = 0;
    hipStream_t stream = nullptr;
    int post_map = 0;  // 0, or a pointwise map applied to every output node (sf_post_map)
    double gamma = 1.4;
    double M[kMaxN * kMaxN];
};

int launch_tensor_apply(const TensorRequest &r);
int launch_tensor_rect(const TensorRequest &r);

// Entropy-projected facet states of 3D Euler states (entropy_kernels.hip).
int launch_entropy_trace(const double *u, double *uf, int64_t E, int n, double gamma, const Operator1D &op,
                         hipStream_t stream);
// Pointwise conserved -> entropy variables (dir 0) or back (dir 1), 5 SoA arrays.
int launch_entropy_map(const double *in, double *out, int64_t count, double gamma, int dir, hipStream_t stream);

// Host modal basis on the nodes of a kind: V[q][k] = L_k(x_q) (orthonormal
// Legendre) and its projection P = V^{-1}.
bool build_basis(int n, int node_kind, double *V, double *P);
// n modes on m >= n nodes: V (m x n) and the L2 projection P (n x m).
bool build_basis_rect(int n, int m, int node_kind, double *V, double *P);

}  // namespace sfhad
