// The surface term (the Remark after Eq. (5)), alone and fused with the
// volume term: sf_block with the facet work as its per-line work.  The
// curvilinear volume term is in curv_kernels.hip.
#include "sf_block.h"

#include <string>

namespace sfhad {
namespace dev {

// ---------------------------------------------------------------------------
// Surface term (the Remark after Eq. (5): the Hadamard product with alpha = 0
// on the facet cubature nodes).  The facet operator of face (m, s) is the
// quadrature-weighted interpolation to xi_m = -1 (s = 0) or +1 (s = 1):
// l_s^T in direction m, W in the others.  Its nonzeros pair each facet node
// with the n volume nodes of the line through it, so the lane that owns line
// L of direction m also owns the two facet nodes t = L of faces (m, 0) and
// (m, 1).  For each it stages the facet state like a volume node (same
// element reference, so log differences stay accurate), evaluates the flux
// with the line's n volume nodes, and accumulates
//     y_face[t] = w_perp sum_k l_s[k] f_m(u_face[t], u_k)   (stored here)
//     t_k      += l_s[k] f_m(u_face[t], u_k)                (line sums; a6
//                                                          applies w_perp)
// 2 d n^d flux evaluations per element.  With VOLUME the line's pairs (a2..a5)
// go into the same line sums too: volume and surface terms in one pass.
template <int N, int DIM, bool VOLUME>
struct SurfaceWork {
    const double *__restrict__ uf;
    double *__restrict__ yf;
    int64_t E;
    kernarg_ptr<double> ell;  // l_s[k] at ell[s * N + k]

    template <int M, int NN, class P, class Op, class R>
    __device__ __forceinline__ void lines(const R *le, int AS, int pbase, int pstride, const Op &op,
                                          const typename P::Consts &K, double gamma, R (&t)[NN][P::NV],
                                          int64_t e, int line, double wperp, const double *ref) const {
        constexpr int T = DIM == 3 ? NN * NN : NN;  // facet nodes per face
        constexpr int NF = 2 * DIM;
        const size_t fstride = (size_t)E * NF * T;
        // fused at n = 8 the two faces run as a loop, one face's staging and
        // sums live at a time (unrolled, that kernel spilled 12 bytes per lane)
        constexpr int kFaceUnroll = (VOLUME && NN == 8) ? 1 : 2;
        // surface alone: both faces' facet states are loaded before the
        // first face's work (one memory latency per line instead of two)
        constexpr bool kBothFirst = !VOLUME;
        double ucb[2][P::NV];
        if constexpr (kBothFirst) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const size_t fidx = ((size_t)e * NF + 2 * M + s) * T + line;
#pragma unroll
                for (int v = 0; v < P::NV; ++v) ucb[s][v] = uf[v * fstride + fidx];
            }
        }
#pragma unroll kFaceUnroll
        for (int s = 0; s < 2; ++s) {
            const size_t fidx = ((size_t)e * NF + 2 * M + s) * T + line;
            double uc[P::NV];
#pragma unroll
            for (int v = 0; v < P::NV; ++v) uc[v] = kBothFirst ? ucb[s][v] : uf[v * fstride + fidx];
            R sa[P::NS];
            P::stage(uc, ref, gamma, sa);
            const typename P::Node A = P::load(sa, 1, 0, M);
            R yfa[P::NV];
#pragma unroll
            for (int k = 0; k < P::NV; ++k) yfa[k] = (R)0;
#pragma unroll
            for (int c = 0; c < NN; ++c) {
                const typename P::Node C = P::load_partner(le, AS, pin(pbase + c * pstride), M);
                R F[P::NV];
                P::pair(A, C, K, F);
                const R l = (R)ell[s * NN + c];
#pragma unroll
                for (int k = 0; k < P::NV; ++k) {
                    yfa[k] = l * F[k] + yfa[k];
                    t[c][k] = l * F[k] + t[c][k];
                }
#pragma unroll
                for (int k = 0; k < P::NV; ++k) {
                    yfa[k] = pin(yfa[k]);
                    t[c][k] = pin(t[c][k]);
                }
            }
#pragma unroll
            for (int k = 0; k < P::NV; ++k) yf[P::out_array(k, M) * fstride + fidx] = (double)yfa[k] * wperp;
        }
        // the volume pairs last: staging a facet state (logarithms,
        // reciprocals) while their sums are live would spill at n = 8
        if constexpr (VOLUME) line_pairs<NN, P, false>(M, le, AS, pbase, pstride, op, K, gamma, t);
    }
};

template <int N>
struct SurfArgs {
    const double *u;
    const double *uf;
    double *yv;
    double *yf;
    int64_t E;
    double gamma;
    OpArg<N> op;
    double ell[2 * N];
};

// at least 3 waves per SIMD (at most 168 VGPRs) up to n = 8, where the
// fused form would otherwise take 188 and run 2; above, 2 (a cap of 168
// would spill the larger line sums)
template <int N, int DIM, class P, bool VOLUME>
__global__ void __launch_bounds__((Geom<N, DIM>::THREADS), (N <= 8 ? 3 : 2))
sf_surface_kernel(const SurfArgs<N>) {
    using L = SfLayout<N, DIM, P>;
    __shared__ double lds[L::LDS_D];
    __shared__ double sref[L::REF_D];
    const auto A = kernel_args<SurfArgs<N>>();
    sf_block<N, DIM, P>(A->u, A->yv, A->E, (int64_t)blockIdx.x * Geom<N, DIM>::EPB, KernargOp<N>{&A->op},
                        A->gamma, lds, sref, SurfaceWork<N, DIM, VOLUME>{A->uf, A->yf, A->E, &A->ell[0]});
}

template <int N, int DIM, class P>
int launch_surface(const VolumeRequest &r) {
    using G = Geom<N, DIM>;
    const int64_t blocks = (r.E + G::EPB - 1) / G::EPB;
    if (blocks > 0x7fffffffLL) {
        set_error("element count too large for one launch");
        return SF_ERR_UNSUPPORTED;
    }
    SurfArgs<N> a;
    a.u = r.u;
    a.uf = r.uf;
    a.yv = r.out;
    a.yf = r.yf;
    a.E = r.E;
    a.gamma = r.gamma;
    fill_op_arg<N>(a.op, r.op);
    for (int i = 0; i < N; ++i) {
        a.ell[i] = r.op.lm[i];
        a.ell[N + i] = r.op.lp[i];
    }
    if (r.mode == kModeVolumeSurface)
        hipLaunchKernelGGL((sf_surface_kernel<N, DIM, P, true>), dim3((unsigned)blocks), dim3(G::THREADS), 0,
                           r.stream, a);
    else
        hipLaunchKernelGGL((sf_surface_kernel<N, DIM, P, false>), dim3((unsigned)blocks), dim3(G::THREADS), 0,
                           r.stream, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("sf_surface_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

template <int DIM, class P, int NMAX>
int dispatch_surface_n(const VolumeRequest &r) {
    switch (r.n) {
#define SF_CASE(NV_)                                                          \
    case NV_:                                                                 \
        if constexpr (NV_ <= NMAX) return launch_surface<NV_, DIM, P>(r);     \
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

int launch_sf_surface(const VolumeRequest &r) {
    using namespace dev;
    if (r.precision != SF_PREC_FP64) {
        set_error("the surface term is built in FP64 only");
        return SF_ERR_UNSUPPORTED;
    }
    switch (r.flux) {
        case SF_FLUX_BURGERS_EC:
            return r.d == 2 ? dispatch_surface_n<2, ScalarFlux<0>, 16>(r) : dispatch_surface_n<3, ScalarFlux<0>, 16>(r);
        case SF_FLUX_PRODUCT:
            return r.d == 2 ? dispatch_surface_n<2, ScalarFlux<2>, 16>(r) : dispatch_surface_n<3, ScalarFlux<2>, 16>(r);
        case SF_FLUX_EULER_CHANDRASHEKAR:
            if (r.d != 3) break;
            return dispatch_surface_n<3, EulerFP64, SF_MAX_N_EULER>(r);
        case SF_FLUX_EULER_CHANDRASHEKAR_PFIX:
            if (r.d != 3) break;
            return dispatch_surface_n<3, EulerPFixFP64, SF_MAX_N_EULER>(r);
        default: break;
    }
    set_error("flux / dimension combination not built");
    return SF_ERR_UNSUPPORTED;
}


}  // namespace sfhad
