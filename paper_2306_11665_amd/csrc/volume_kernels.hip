// Sum-factorized volume kernels (Eq. (3) with the coefficients of Eq. (5)):
// the standalone launch of sf_block with the volume pairs as its line work,
// for every (n, d, flux, precision) built.  The serving kernels, which run
// the same blocks for batches of requests, are in serve_kernels.hip.
#include "sf_block.h"

#include <string>
#include <type_traits>

namespace sfhad {
namespace dev {

template <class P, class = void>
struct PressureFix : std::false_type {};
template <class P>
struct PressureFix<P, std::void_t<decltype(P::PRESSURE_FIX)>> : std::bool_constant<P::PRESSURE_FIX> {};

// Launch shape of the standalone kernel: the 3D Euler flux takes
// euler_volume_shape, the scalar fluxes the grouped mapping.
template <int N, int DIM, class P>
constexpr VolumeShape volume_shape() {
    return (DIM == 3 && P::NV == 5) ? euler_volume_shape(N, sizeof(typename P::Real) == 8, PressureFix<P>::value)
                                    : VolumeShape{0, 1, N <= 8, false};
}

template <int N, int DIM, class P>
__global__ void __launch_bounds__((Geom<N, DIM, volume_shape<N, DIM, P>().fe>::THREADS),
                                  (volume_shape<N, DIM, P>().min_waves))
sf_volume_kernel(const VolArgs<N> args) {
    constexpr int FE = volume_shape<N, DIM, P>().fe;
    using L = SfLayout<N, DIM, P, FE>;
    __shared__ double lds[L::LDS_D];
    __shared__ double sref[L::REF_D];
    const int64_t e0 = (int64_t)blockIdx.x * Geom<N, DIM, FE>::EPB;
    using Work = VolumeWorkT<volume_shape<N, DIM, P>().ahead>;
    constexpr bool OWN = volume_shape<N, DIM, P>().own_ref;
    if constexpr (N <= 9) {
        sf_block<N, DIM, P, FE, OWN>(args.u, args.out, args.E, e0, ParamOp<N>{args.op}, args.gamma, lds, sref,
                                     Work{});
    } else {
        const auto A = kernel_args<VolArgs<N>>();
        sf_block<N, DIM, P, FE, OWN>(A->u, A->out, A->E, e0, KernargOp<N>{&A->op}, A->gamma, lds, sref, Work{});
    }
}

template <int N>
VolArgs<N> make_args(const VolumeRequest &r) {
    VolArgs<N> a;
    a.u = r.u;
    a.out = r.out;
    a.E = r.E;
    a.gamma = r.gamma;
    fill_op_arg<N>(a.op, r.op);
    return a;
}

template <int N, int DIM, class P>
int launch_sf(const VolumeRequest &r) {
    using G = Geom<N, DIM, volume_shape<N, DIM, P>().fe>;
    const int64_t blocks = (r.E + G::EPB - 1) / G::EPB;
    if (blocks > 0x7fffffffLL) {
        set_error("element count too large for one launch");
        return SF_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL((sf_volume_kernel<N, DIM, P>), dim3((unsigned)blocks), dim3(G::THREADS), 0,
                       r.stream, make_args<N>(r));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("sf_volume_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

// Dispatch on n for a fixed (DIM, policy); n range [2, NMAX].
template <int DIM, class P, int NMAX>
int dispatch_n(const VolumeRequest &r) {
    switch (r.n) {
#define SF_CASE(NV_)                                                       \
    case NV_:                                                              \
        if constexpr (NV_ <= NMAX) return launch_sf<NV_, DIM, P>(r);       \
        break;
        SF_CASE(2) SF_CASE(3) SF_CASE(4) SF_CASE(5) SF_CASE(6) SF_CASE(7) SF_CASE(8) SF_CASE(9)
        SF_CASE(10) SF_CASE(11) SF_CASE(12) SF_CASE(13) SF_CASE(14) SF_CASE(15) SF_CASE(16)
#undef SF_CASE
        default: break;
    }
    set_error("n outside the built range");
    return SF_ERR_UNSUPPORTED;
}

}  // namespace dev

// The build compiles this file twice: SF_VOLUME_PART 1 instantiates the FP64
// and scalar-flux kernels and the dispatch, 2 the FP32-split kernels, each
// with its own scheduling options (the FP32-split form runs faster with
// another schedule); without SF_VOLUME_PART one object holds both.
int launch_sf_volume_fp32(const VolumeRequest &r);

#if !defined(SF_VOLUME_PART) || SF_VOLUME_PART == 2
int launch_sf_volume_fp32(const VolumeRequest &r) {
    return dev::dispatch_n<3, dev::EulerFP32Split, SF_MAX_N_EULER>(r);
}
#endif

#if !defined(SF_VOLUME_PART) || SF_VOLUME_PART == 1
int launch_sf_volume(const VolumeRequest &r) {
    using namespace dev;
    if (r.precision == SF_PREC_FP32_SPLIT) {
        if (r.flux == SF_FLUX_EULER_CHANDRASHEKAR && r.d == 3) return launch_sf_volume_fp32(r);
        set_error("the FP32-split form is built for the 3D Euler flux only");
        return SF_ERR_UNSUPPORTED;
    }
    switch (r.flux) {
        case SF_FLUX_BURGERS_EC:
            return r.d == 2 ? dispatch_n<2, ScalarFlux<0>, 16>(r) : dispatch_n<3, ScalarFlux<0>, 16>(r);
        case SF_FLUX_PRODUCT:
            return r.d == 2 ? dispatch_n<2, ScalarFlux<2>, 16>(r) : dispatch_n<3, ScalarFlux<2>, 16>(r);
        case SF_FLUX_EULER_CHANDRASHEKAR:
            if (r.d != 3) break;
            return dispatch_n<3, EulerFP64, SF_MAX_N_EULER>(r);
        case SF_FLUX_EULER_CHANDRASHEKAR_PFIX:
            if (r.d != 3) break;
            return dispatch_n<3, EulerPFixFP64, SF_MAX_N_EULER>(r);
        default: break;
    }
    set_error("flux / dimension combination not built");
    return SF_ERR_UNSUPPORTED;
}
#endif

}  // namespace sfhad
