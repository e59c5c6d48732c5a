// Dense O(n^(2d)) volume kernel: the Hadamard product of Eq. (1)/(3) taken
// literally, the speed baseline of the sum-factorized kernels.
//
// One workgroup per element.  The per-node quantities are staged in LDS
// exactly as in the sum-factorized kernel; then each thread owns row nodes
// i and, for every direction m and every column node j of the element,
// forms A_m[i][j] = Q[i_m][j_m] * prod_{k != m} (i_k == j_k ? w[i_k] : 0)
// and adds A_m[i][j] f_m(u_i, u_j) -- all n^d x n^d pairs, zero coefficients
// included, each direction's flux evaluated on its own (no sharing of the
// logarithmic means across directions).  Column data are LDS broadcasts.
#include "kernels_common.h"
#include "sfhad_internal.h"

namespace sfhad {
namespace dev {

template <int N, int DIM>
struct DenseGeom {
    static constexpr int NODES = DIM == 3 ? N * N * N : N * N;
    static constexpr int R64 = ((NODES + 63) / 64) * 64;
    static constexpr int THREADS = R64 < 512 ? R64 : 512;
};

template <int N, int DIM, class P>
__global__ void __launch_bounds__((DenseGeom<N, DIM>::THREADS))
dense_volume_kernel(const VolArgs<N>) {
    using G = DenseGeom<N, DIM>;
    const auto A = kernel_args<VolArgs<N>>();
    const double *__restrict__ u = A->u;
    double *__restrict__ out = A->out;
    const int64_t E = A->E;
    const double gamma = A->gamma;
    constexpr int NODES = G::NODES;
    __shared__ double lds[P::NS * NODES];
    __shared__ double sQ[N * N];
    __shared__ double sw[N];

    const int tid = threadIdx.x;
    const int64_t e = blockIdx.x;
    const size_t vstride = (size_t)E * NODES;
    const size_t gbase = (size_t)e * NODES;

    for (int i = tid; i < N * N; i += G::THREADS) sQ[i] = A->op.Q[i];
    for (int i = tid; i < N; i += G::THREADS) sw[i] = A->op.w[i];
    constexpr int NREF = P::NREF > 0 ? P::NREF : 1;
    __shared__ double sref[NREF];
    if (P::NREF > 0) {
        if (tid == 0) {
            double uc[P::NV];
#pragma unroll
            for (int v = 0; v < P::NV; ++v) uc[v] = u[v * vstride + gbase];
            P::make_ref(uc, gamma, sref);
        }
        __syncthreads();
    }
    for (int i = tid; i < NODES; i += G::THREADS) {
        double uc[P::NV], s[P::NS];
#pragma unroll
        for (int v = 0; v < P::NV; ++v) uc[v] = u[v * vstride + gbase + i];
        P::stage(uc, sref, gamma, s);
#pragma unroll
        for (int k = 0; k < P::NS; ++k) lds[k * NODES + i] = s[k];
    }
    __syncthreads();

    const typename P::Consts K = P::consts(0.5 / (gamma - 1.0));
    for (int i = tid; i < NODES; i += G::THREADS) {
        int di[3] = {i % N, (i / N) % N, DIM == 3 ? i / (N * N) : 0};
        double y[P::NV];
#pragma unroll
        for (int v = 0; v < P::NV; ++v) y[v] = 0.0;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            const typename P::Node I = P::load(lds, NODES, i, m);
            double acc[P::NV];
#pragma unroll
            for (int k = 0; k < P::NV; ++k) acc[k] = 0.0;
            for (int j = 0; j < NODES; ++j) {
                const int dj[3] = {j % N, (j / N) % N, DIM == 3 ? j / (N * N) : 0};
                double a = sQ[di[m] * N + dj[m]];
#pragma unroll
                for (int k = 0; k < DIM; ++k)
                    if (k != m) a *= (di[k] == dj[k]) ? sw[di[k]] : 0.0;
                const typename P::Node J = P::load(lds, NODES, j, m);
                double F[P::NV];
                P::pair(I, J, K, F);
#pragma unroll
                for (int k = 0; k < P::NV; ++k) acc[k] = __builtin_fma(a, F[k], acc[k]);
            }
#pragma unroll
            for (int k = 0; k < P::NV; ++k) y[P::out_array(k, m)] += acc[k];
        }
#pragma unroll
        for (int v = 0; v < P::NV; ++v) out[v * vstride + gbase + i] = y[v];
    }
}

template <int N>
VolArgs<N> make_dense_args(const VolumeRequest &r) {
    VolArgs<N> a;
    a.u = r.u;
    a.out = r.out;
    a.E = r.E;
    a.gamma = r.gamma;
    fill_op_arg<N>(a.op, r.op);
    return a;
}

template <int N, int DIM, class P>
int launch_dense(const VolumeRequest &r) {
    using G = DenseGeom<N, DIM>;
    if (r.E > 0x7fffffffLL) {
        set_error("element count too large for one launch");
        return SF_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL((dense_volume_kernel<N, DIM, P>), dim3((unsigned)r.E), dim3(G::THREADS), 0,
                       r.stream, make_dense_args<N>(r));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("dense_volume_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

template <int DIM, class P, int NMAX>
int dispatch_dense_n(const VolumeRequest &r) {
    switch (r.n) {
#define SF_CASE(NV_)                                                        \
    case NV_:                                                               \
        if constexpr (NV_ <= NMAX) return launch_dense<NV_, DIM, P>(r);     \
        break;
        SF_CASE(2) SF_CASE(3) SF_CASE(4) SF_CASE(5) SF_CASE(6) SF_CASE(7) SF_CASE(8) SF_CASE(9)
        SF_CASE(10) SF_CASE(11) SF_CASE(12) SF_CASE(13) SF_CASE(14) SF_CASE(15) SF_CASE(16)
#undef SF_CASE
        default: break;
    }
    set_error("n outside the built dense range");
    return SF_ERR_UNSUPPORTED;
}

}  // namespace dev

int launch_dense_volume(const VolumeRequest &r) {
    using namespace dev;
    if (r.precision != SF_PREC_FP64) {
        set_error("the dense path is built in FP64 only");
        return SF_ERR_UNSUPPORTED;
    }
    switch (r.flux) {
        case SF_FLUX_BURGERS_EC:
            return r.d == 2 ? dispatch_dense_n<2, ScalarFlux<0>, 16>(r)
                            : dispatch_dense_n<3, ScalarFlux<0>, 16>(r);
        case SF_FLUX_PRODUCT:
            return r.d == 2 ? dispatch_dense_n<2, ScalarFlux<2>, 16>(r)
                            : dispatch_dense_n<3, ScalarFlux<2>, 16>(r);
        case SF_FLUX_EULER_CHANDRASHEKAR:
            if (r.d != 3) break;
            return dispatch_dense_n<3, EulerFP64, SF_MAX_N_EULER>(r);
        case SF_FLUX_EULER_CHANDRASHEKAR_PFIX:
            if (r.d != 3) break;
            return dispatch_dense_n<3, EulerPFixFP64, SF_MAX_N_EULER>(r);
        default: break;
    }
    set_error("flux / dimension combination not built");
    return SF_ERR_UNSUPPORTED;
}

}  // namespace sfhad
