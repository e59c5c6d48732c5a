// The curvilinear (metric-averaged) volume term: sf_block with the
// metric-averaged flux policies.
#include "sf_block.h"

#include <string>

namespace sfhad {
namespace dev {

// ---------------------------------------------------------------------------
// Curvilinear elements: the volume kernel with the metric-averaged flux
// (EulerCurvFP64, or EulerCurvPFixFP64 with the pressure fix); the 9 metric
// terms per node are staged with the state.
template <int N>
struct CurvArgs {
    const double *u;
    const double *Ja;
    double *out;
    int64_t E;
    double gamma;
    OpArg<N> op;
};

template <int N, class P>
__global__ void __launch_bounds__((Geom<N, 3>::THREADS))
sf_curv_kernel(const CurvArgs<N>) {
    using L = SfLayout<N, 3, P>;
    __shared__ double lds[L::LDS_D];
    __shared__ double sref[L::REF_D];
    const auto A = kernel_args<CurvArgs<N>>();
    sf_block<N, 3, P>(A->u, A->out, A->E, (int64_t)blockIdx.x * Geom<N, 3>::EPB, KernargOp<N>{&A->op}, A->gamma,
                      lds, sref, VolumeWork{}, A->Ja);
}

template <int N>
int launch_curv(const VolumeRequest &r) {
    using G = Geom<N, 3>;
    const int64_t blocks = (r.E + G::EPB - 1) / G::EPB;
    if (blocks > 0x7fffffffLL) {
        set_error("element count too large for one launch");
        return SF_ERR_UNSUPPORTED;
    }
    CurvArgs<N> a;
    a.u = r.u;
    a.Ja = r.aux;
    a.out = r.out;
    a.E = r.E;
    a.gamma = r.gamma;
    fill_op_arg<N>(a.op, r.op);
    if (r.flux == SF_FLUX_EULER_CHANDRASHEKAR_PFIX)
        hipLaunchKernelGGL((sf_curv_kernel<N, EulerCurvPFixFP64>), dim3((unsigned)blocks), dim3(G::THREADS), 0,
                           r.stream, a);
    else
        hipLaunchKernelGGL((sf_curv_kernel<N, EulerCurvFP64>), dim3((unsigned)blocks), dim3(G::THREADS), 0,
                           r.stream, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("sf_curv_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

}  // namespace dev

int launch_sf_curvilinear(const VolumeRequest &r) {
    using namespace dev;
    switch (r.n) {
        case 2: return launch_curv<2>(r);
        case 3: return launch_curv<3>(r);
        case 4: return launch_curv<4>(r);
        case 5: return launch_curv<5>(r);
        case 6: return launch_curv<6>(r);
        case 7: return launch_curv<7>(r);
        case 8: return launch_curv<8>(r);
        case 9: return launch_curv<9>(r);
        case 10: return launch_curv<10>(r);
        default: break;
    }
    set_error("the curvilinear kernel is built for 2 <= n <= 10");
    return SF_ERR_UNSUPPORTED;
}

}  // namespace sfhad
