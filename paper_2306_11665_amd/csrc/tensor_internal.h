// Internal declarations of the basis-transformation path (tensor_kernels.hip,
// operators.cpp, capi.cpp).
#pragma once

#include "sfhad_internal.h"

namespace sfhad {

// A validated sf_tensor_apply request: out_e = (M (x) ... (x) M) in_e for
// E elements of nvar variables (slab v * E + e holds n^d doubles).
struct TensorRequest {
    const double *in = nullptr;
    double *out = nullptr;
    int64_t E = 0;
    int n = 0;
    int d = 0;
    int nvar = 0;
    hipStream_t stream = nullptr;
    double M[kMaxN * kMaxN];
};

int launch_tensor_apply(const TensorRequest &r);

// Entropy-projected facet states of 3D Euler states (entropy_kernels.hip).
int launch_entropy_trace(const double *u, double *uf, int64_t E, int n, double gamma, const Operator1D &op,
                         hipStream_t stream);

// Host modal basis on the nodes of a kind: V[q][k] = L_k(x_q) (orthonormal
// Legendre) and its projection P = V^{-1}.
bool build_basis(int n, int node_kind, double *V, double *P);

}  // namespace sfhad
