// Entropy-projected facet states for the surface term (3D Euler, FP64):
//     u_face[t] = u( sum_k l_s[k] v(u_k) )
// over the n nodes u_k of the line through facet node t of face (m, s): the
// conserved variables of the facet-interpolated entropy variables (with as
// many nodes as modes per direction the L2 projection of v is v itself, so
// this is u(V_f P v(u))).  v = dU/du for U = -rho s/(gamma - 1),
// s = ln p - gamma ln rho:
//     v = ((gamma - s)/(gamma - 1) - rho |vel|^2/(2p), rho vel/p, -rho/p),
// and its inverse from rho/p = -v_4: vel = v_1..3/(rho/p),
// s = gamma - (gamma - 1)(v_0 + (rho/p)|vel|^2/2),
// rho = exp((s + ln(rho/p))/(1 - gamma)), p = rho/(rho/p).
//
// One workgroup per element: the nodal entropy variables go to LDS (one
// padded array per component), then each thread takes facet nodes in the
// output order (face-major, t fastest: coalesced stores) and interpolates
// along its line.  Moves 8 B x 5 x (n^3 + 6 n^2) per element; the maps are
// the shared ones of entropy_maps.h (own logarithm and exponential, about one
// ulp; quotients are products with a refined reciprocal), the 1/(gamma - 1)
// factors one reciprocal per thread.
#include "entropy_maps.h"
#include "kernels_common.h"
#include "sfhad_internal.h"

namespace sfhad {
namespace dev {

constexpr int kTraceThreads = 128;  // n = 8: 512 nodes and 384 facet nodes, no idle lane

template <int N>
struct TraceArgs {
    const double *u;
    double *uf;
    int64_t E;
    double gamma;
    double lm[N];
    double lp[N];
};

template <int N>
__device__ __forceinline__ int trace_node(int t, int k, int m) {
    if (m == 0) return k + N * t;                          // t = iy + n iz
    if (m == 1) return (t % N) + N * k + N * N * (t / N);  // t = ix + n iz
    return t + N * N * k;                                  // t = ix + n iy
}

template <int N>
__global__ void __launch_bounds__(kTraceThreads) entropy_trace_kernel(const TraceArgs<N>) {
    constexpr int NODES = N * N * N, T = N * N, NF = 6, PAD = NODES + NODES / N;
    __shared__ double sv[5 * PAD];
    const auto A = kernel_args<TraceArgs<N>>();
    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const double g = A->gamma;
    const double igm1 = uniform_f64(1.0 / (g - 1.0));
    const size_t vs = (size_t)A->E * NODES, base = (size_t)e * NODES;
    // every load of the element's state is issued before the first
    // conversion (1.10x at n = 8, 1.19x at n = 10 against converting node by
    // node as the loads return)
    constexpr int NPT = (NODES + kTraceThreads - 1) / kTraceThreads;
    double uc[NPT][5];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int i = tid + j * kTraceThreads;
        if (i < NODES) {
#pragma unroll
            for (int c = 0; c < 5; ++c) uc[j][c] = A->u[c * vs + base + i];
        }
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int i = tid + j * kTraceThreads;
        if (i >= NODES) break;
        double y[5];
        entropy_from_conserved(uc[j], g, igm1, y);
        const int li = i + i / N;
#pragma unroll
        for (int c = 0; c < 5; ++c) sv[c * PAD + li] = y[c];
    }
    __syncthreads();
    const size_t fs = (size_t)A->E * NF * T;
    const size_t fbase = (size_t)e * NF * T;
    for (int j = tid; j < NF * T; j += kTraceThreads) {
        const int f = j / T, t = j - f * T;
        const int m = f >> 1;
        double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double l = (f & 1) ? A->lp[k] : A->lm[k];
            const int nd = trace_node<N>(t, k, m);
            const int li = nd + nd / N;
#pragma unroll
            for (int c = 0; c < 5; ++c) v[c] = __builtin_fma(l, sv[c * PAD + li], v[c]);
        }
        double y[5];
        conserved_from_entropy(v, g, igm1, y);
#pragma unroll
        for (int c = 0; c < 5; ++c) A->uf[c * fs + fbase + j] = y[c];
    }
}

template <int N>
int launch_trace(const double *u, double *uf, int64_t E, double gamma, const Operator1D &op, hipStream_t st) {
    if (E > 0x7fffffffLL) {
        set_error("element count too large for one launch");
        return SF_ERR_UNSUPPORTED;
    }
    TraceArgs<N> a;
    a.u = u;
    a.uf = uf;
    a.E = E;
    a.gamma = gamma;
    for (int i = 0; i < N; ++i) {
        a.lm[i] = op.lm[i];
        a.lp[i] = op.lp[i];
    }
    hipLaunchKernelGGL((entropy_trace_kernel<N>), dim3((unsigned)E), dim3(kTraceThreads), 0, st, a);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("entropy_trace_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

// Pointwise maps over SoA arrays of `count` states (5 arrays of count
// doubles): conserved -> entropy variables (dir = 0) or back (dir = 1).
// Grid-stride, coalesced; for composing the entropy projection with the
// basis transformation (u(V P v(u)) on any node set).
__global__ void __launch_bounds__(256) entropy_map_kernel(const double *__restrict__ in, double *__restrict__ out,
                                                         int64_t count, double g, int dir) {
    const double igm1 = 1.0 / (g - 1.0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x[5] = {in[i], in[count + i], in[2 * count + i], in[3 * count + i], in[4 * count + i]};
        double y[5];
        if (dir == 0)
            entropy_from_conserved(x, g, igm1, y);
        else
            conserved_from_entropy(x, g, igm1, y);
#pragma unroll
        for (int c = 0; c < 5; ++c) out[c * count + i] = y[c];
    }
}

}  // namespace dev

int launch_entropy_trace(const double *u, double *uf, int64_t E, int n, double gamma, const Operator1D &op,
                         hipStream_t st) {
    using namespace dev;
    switch (n) {
        case 2: return launch_trace<2>(u, uf, E, gamma, op, st);
        case 3: return launch_trace<3>(u, uf, E, gamma, op, st);
        case 4: return launch_trace<4>(u, uf, E, gamma, op, st);
        case 5: return launch_trace<5>(u, uf, E, gamma, op, st);
        case 6: return launch_trace<6>(u, uf, E, gamma, op, st);
        case 7: return launch_trace<7>(u, uf, E, gamma, op, st);
        case 8: return launch_trace<8>(u, uf, E, gamma, op, st);
        case 9: return launch_trace<9>(u, uf, E, gamma, op, st);
        case 10: return launch_trace<10>(u, uf, E, gamma, op, st);
        case 11: return launch_trace<11>(u, uf, E, gamma, op, st);
        case 12: return launch_trace<12>(u, uf, E, gamma, op, st);
        case 13: return launch_trace<13>(u, uf, E, gamma, op, st);
        default: break;
    }
    set_error("the entropy trace is built for 2 <= n <= 13");
    return SF_ERR_UNSUPPORTED;
}

int launch_entropy_map(const double *in, double *out, int64_t count, double gamma, int dir, hipStream_t st) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(dev::entropy_map_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, out, count, gamma, dir);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("entropy_map_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

}  // namespace sfhad
