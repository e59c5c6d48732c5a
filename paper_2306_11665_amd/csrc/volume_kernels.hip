// Sum-factorized volume kernels (Eq. (3) with the coefficients of Eq. (5)).
//
// One workgroup per block of EPB elements; d groups of LPD lanes, group m
// handling every line of direction m of the block's elements, one line per
// lane (at n = 8 in 3D: one element, 3 waves of 64 lanes, 64 lines each).
//
//   a1  stage:   coalesced SoA loads of the conserved state, conversion to
//                the flux's per-node quantities, stored in LDS;
//   a2  lines:   the lane's line = padded LDS base + a * stride (Algorithm 1
//                as index arithmetic, nothing materialized);
//   a3  coeffs:  Q[a][c] from the kernel arguments (scalar registers),
//                w_perp once per line (Algorithm 2's values, on the fly);
//   a4  flux:    every unordered pair (a < c) once plus the n diagonal
//                physical fluxes;
//   a5  reduce:  t_a += Q[a][c] F, t_c += Q[c][a] F in registers;
//   a6  sum:     t * w_perp summed over the d directions in FP64 in LDS in the
//                fixed order m = 0, 1, 2 (bit-reproducible), then coalesced
//                stores.
//   a7  the FP32-split form is the same kernel with the EulerFP32Split policy
//                (FP32 inputs, flux and line sums; FP64 direction sum).
#include "kernels_common.h"
#include "sfhad_internal.h"

#include <algorithm>
#include <cstring>

namespace sfhad {
namespace dev {

// a2..a5 for one line: every unordered pair (a < c) once plus the diagonal,
// accumulated into t.  The loads of the stored arrays are rotated into the
// frame of direction M.
template <int N, class P, int M, class Op>
__device__ __forceinline__ void line_pairs(const typename P::Real *le, int AS, int pbase, int pstride,
                                           const Op &op, const typename P::Consts &K, double gamma,
                                           typename P::Real (&t)[N][P::NV]) {
    using R = typename P::Real;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const typename P::Node A = P::load(le, AS, pin(pbase + a * pstride), M);
        R F[P::NV];
        P::diag(A, gamma, F);
        const R qaa = (R)op.q(a * N + a);
#pragma unroll
        for (int k = 0; k < P::NV; ++k) t[a][k] = qaa * F[k] + t[a][k];
#pragma unroll
        for (int c = a + 1; c < N; ++c) {
            // re-read node c from LDS for every pair: an opaque index stops
            // the compiler from keeping the whole line live in registers
            const typename P::Node C = P::load_partner(le, AS, pin(pbase + c * pstride), M);
            P::pair(A, C, K, F);
            const R qac = (R)op.q(a * N + c), qca = (R)op.q(c * N + a);
#pragma unroll
            for (int k = 0; k < P::NV; ++k) {
                t[a][k] = qac * F[k] + t[a][k];
                t[c][k] = qca * F[k] + t[c][k];
            }
            // one pair in flight at a time: its sums complete here, before
            // the next pair's loads (ordered after this fence) are issued
#pragma unroll
            for (int k = 0; k < P::NV; ++k) {
                t[a][k] = pin(t[a][k]);
                t[c][k] = pin(t[c][k]);
            }
        }
    }
}

// Distance between two stored arrays, in elements of size `bytes`: at least
// `base`, padded so that consecutive arrays start 8 banks apart (the
// unpadded n = 8 layout puts every array on the same bank).
template <int bytes>
constexpr int array_stride(int base) {
    int as = base;
    while (((as * bytes / 4) % 32) != 8) ++as;
    return as;
}

// LDS needed by one block of the sum-factorized kernel: the staged inputs
// (NS arrays of Real) and, after the compute phase, the FP64 outputs (NV
// arrays of doubles, same stride) share the buffer.
template <int N, int DIM, class P>
struct SfLayout {
    using G = Geom<N, DIM>;
    using R = typename P::Real;
    static constexpr int AS = array_stride<(int)sizeof(R)>(G::EPB * G::PADN);  // array distance (elements)
    static constexpr int IN_D = (P::NS * AS * (int)sizeof(R) + 7) / 8;
    static constexpr int OUT_D = P::NV * AS;
    static constexpr int LDS_D = IN_D > OUT_D ? IN_D : OUT_D;  // doubles
    static constexpr int NREF = P::NREF > 0 ? P::NREF : 1;
    static constexpr int REF_D = G::EPB * NREF;                // doubles
};

// The 1D operator, read from the kernel arguments (standalone launches) or
// from a device table (the serving kernel).  Both give the same values.
template <int N>
struct KernargOp {
    kernarg_ptr<OpArg<N>> a;
    __device__ double q(int i) const { return a->Q[i]; }
    __device__ double w(int i) const { return a->w[i]; }
};

// The same through a reference to the by-value parameter: for the small
// argument blocks (n <= 9) clang keeps it in the argument segment, and the
// kernels come out slightly faster this way.
template <int N>
struct ParamOp {
    const OpArg<N> &a;
    __device__ double q(int i) const { return a.Q[i]; }
    __device__ double w(int i) const { return a.w[i]; }
};

struct TableOp {
    const double *__restrict__ Q;
    const double *__restrict__ W;
    // the base is made opaque at every read so that the (scalar) loads stay
    // next to their use instead of being hoisted and held in registers
    __device__ double q(int i) const {
        const double *p = Q;
        asm volatile("" : "+s"(p));
        return p[i];
    }
    __device__ double w(int i) const { return W[i]; }
};

// The per-line work of a block.  VolumeWork is a2..a5 (every pair of the
// line); SurfaceWork is the facet part of the surface term (below);
// VolumeSurfaceWork does both into the same line sums.
struct VolumeWork {
    template <int M, int N, class P, class Op, class R>
    __device__ __forceinline__ void lines(const R *le, int AS, int pbase, int pstride, const Op &op,
                                          const typename P::Consts &K, double gamma, R (&t)[N][P::NV], int64_t,
                                          int, double, const double *) const {
        line_pairs<N, P, M>(le, AS, pbase, pstride, op, K, gamma, t);
    }
};

// One block of EPB elements starting at element e0 of an E-element mesh:
// steps a1..a6 with the line work of `work`.  lds holds SfLayout::LDS_D
// doubles, sref SfLayout::REF_D.
template <int N, int DIM, class P, class Op, class Work = VolumeWork>
__device__ __forceinline__ void sf_block(const double *__restrict__ u, double *__restrict__ out, int64_t E,
                                         int64_t e0, const Op &op, double gamma, double *lds, double *sref,
                                         const Work &work = Work{}, const double *__restrict__ aux = nullptr) {
    using G = Geom<N, DIM>;
    using L = SfLayout<N, DIM, P>;
    using R = typename P::Real;
    constexpr int AS = L::AS;
    constexpr int NREF = L::NREF;
    R *lin = reinterpret_cast<R *>(lds);  // staged inputs: NS arrays of type R
    double *lout = lds;                   // outputs: NV arrays of doubles

    const int tid = threadIdx.x;
    const int nel = (int)((E - e0) < G::EPB ? (E - e0) : G::EPB);
    const int nvalid = nel * G::NODES;
    const size_t vstride = (size_t)E * G::NODES;
    const size_t gbase = (size_t)e0 * G::NODES;

    // a1: per-element reference values (from each element's first node), then
    // stage the block's nodes.
    if (P::NREF > 0) {
        if (tid < nel) {
            double uc[P::NV];
#pragma unroll
            for (int v = 0; v < P::NV; ++v) uc[v] = u[v * vstride + gbase + (size_t)tid * G::NODES];
            P::make_ref(uc, gamma, sref + tid * NREF);
        }
        __syncthreads();
    }
    // every load of the staging pass is issued before any conversion
    constexpr int SPT = (G::EPB * G::NODES + G::THREADS - 1) / G::THREADS;  // nodes per thread
    double uc[SPT][P::NV + P::NX];  // conserved variables, then P::NX extra inputs from aux
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int i = tid + k * G::THREADS;
        if (i < nvalid) {
#pragma unroll
            for (int v = 0; v < P::NV; ++v) uc[k][v] = u[v * vstride + gbase + i];
#pragma unroll
            for (int x = 0; x < P::NX; ++x) uc[k][P::NV + x] = aux[x * vstride + gbase + i];
        }
    }
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int i = tid + k * G::THREADS;
        if (i < nvalid) {
            R s[P::NS];
            P::stage(uc[k], sref + (i / G::NODES) * NREF, gamma, s);
            const int el = i / G::NODES, node = i - el * G::NODES;
            const int li = el * G::PADN + G::pidx(node);
#pragma unroll
            for (int q = 0; q < P::NS; ++q) lin[q * AS + li] = s[q];
        }
    }
    __syncthreads();

    // a2..a5: one line per lane.
    const int m = tid / G::LPD;
    const int r = tid - m * G::LPD;
    const int el = r / G::LINES;
    const int line = r - el * G::LINES;
    const bool active = el < nel;
    int pbase, pstride, q0, q1;
    line_geometry<N, DIM>(m, line, pbase, pstride, q0, q1);
    const double wperp = DIM == 3 ? op.w(q0) * op.w(q1) : op.w(q0);
    const typename P::Consts K = P::consts(0.5 / (gamma - 1.0));
    const R *le = lin + el * G::PADN;

    R t[N][P::NV];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int k = 0; k < P::NV; ++k) t[a][k] = (R)0;

    if (active) {
        // m is uniform per wave; one instantiation per direction turns the
        // rotated array offsets into immediates
        const int64_t e = e0 + el;
        const double *ref = sref + el * NREF;
        if (m == 0)
            work.template lines<0, N, P>(le, AS, pbase, pstride, op, K, gamma, t, e, line, wperp, ref);
        else if (DIM == 2 || m == 1)
            work.template lines<1, N, P>(le, AS, pbase, pstride, op, K, gamma, t, e, line, wperp, ref);
        else
            work.template lines<2, N, P>(le, AS, pbase, pstride, op, K, gamma, t, e, line, wperp, ref);
    }
    __syncthreads();  // every lane is done reading the staged inputs

    // a6: FP64 direction sum in the fixed order m = 0, 1, ..., d-1 (bit
    // reproducible): the first directions accumulate in LDS (the output
    // arrays reuse the input space), the last adds its own sums to the LDS
    // total and stores the result (for fixed a, the lanes of the last
    // direction cover consecutive nodes: coalesced).
    double *lo = lout + el * G::PADN;
    const size_t obase = gbase + (size_t)el * G::NODES;
#pragma unroll
    for (int mm = 0; mm < DIM; ++mm) {
        if (m == mm && active) {
            const int nstride = DIM == 3 ? N * N : N;  // node stride of the last direction
            const int nbase = DIM == 3 ? q0 + N * q1 : q0;
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const int idx = pbase + a * pstride;
#pragma unroll
                for (int k = 0; k < P::NV; ++k) {
                    double *dst = lo + P::out_array(k, m) * AS + idx;
                    const double val = (double)t[a][k] * wperp;
                    if (mm == 0)
                        *dst = val;
                    else if (mm < DIM - 1)
                        *dst = *dst + val;
                    else
                        out[P::out_array(k, m) * vstride + obase + nbase + a * nstride] = *dst + val;
                }
            }
        }
        if (mm < DIM - 1) __syncthreads();
    }
}

template <int N, int DIM, class P>
__global__ void __launch_bounds__((Geom<N, DIM>::THREADS))
sf_volume_kernel(const VolArgs<N> args) {
    using L = SfLayout<N, DIM, P>;
    __shared__ double lds[L::LDS_D];
    __shared__ double sref[L::REF_D];
    const int64_t e0 = (int64_t)blockIdx.x * Geom<N, DIM>::EPB;
    if constexpr (N <= 9) {
        sf_block<N, DIM, P>(args.u, args.out, args.E, e0, ParamOp<N>{args.op}, args.gamma, lds, sref);
    } else {
        const auto A = kernel_args<VolArgs<N>>();
        sf_block<N, DIM, P>(A->u, A->out, A->E, e0, KernargOp<N>{&A->op}, A->gamma, lds, sref);
    }
}

template <int N>
VolArgs<N> make_args(const VolumeRequest &r) {
    VolArgs<N> a;
    a.u = r.u;
    a.out = r.out;
    a.E = r.E;
    a.gamma = r.gamma;
    for (int i = 0; i < N * N; ++i) a.op.Q[i] = r.op.Q[i];
    for (int i = 0; i < N; ++i) a.op.w[i] = r.op.w[i];
    return a;
}

template <int N, int DIM, class P>
int launch_sf(const VolumeRequest &r) {
    using G = Geom<N, DIM>;
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
// go into the same line sums first: volume and surface terms in one pass.
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
        if constexpr (VOLUME) line_pairs<NN, P, M>(le, AS, pbase, pstride, op, K, gamma, t);
        constexpr int T = DIM == 3 ? NN * NN : NN;  // facet nodes per face
        constexpr int NF = 2 * DIM;
        const size_t fstride = (size_t)E * NF * T;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const size_t fidx = ((size_t)e * NF + 2 * M + s) * T + line;
            double uc[P::NV];
#pragma unroll
            for (int v = 0; v < P::NV; ++v) uc[v] = uf[v * fstride + fidx];
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

// at least 3 waves per SIMD (at most 168 VGPRs): the fused form would
// otherwise take 188 at n = 8 and run 2
template <int N, int DIM, class P, bool VOLUME>
__global__ void __launch_bounds__((Geom<N, DIM>::THREADS), 3)
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
    for (int i = 0; i < N * N; ++i) a.op.Q[i] = r.op.Q[i];
    for (int i = 0; i < N; ++i) {
        a.op.w[i] = r.op.w[i];
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

// ---------------------------------------------------------------------------
// Curvilinear elements: the volume kernel with the metric-averaged flux
// (EulerCurvFP64); the 9 metric terms per node are staged with the state.
template <int N>
struct CurvArgs {
    const double *u;
    const double *Ja;
    double *out;
    int64_t E;
    double gamma;
    OpArg<N> op;
};

template <int N>
__global__ void __launch_bounds__((Geom<N, 3>::THREADS))
sf_curv_kernel(const CurvArgs<N>) {
    using L = SfLayout<N, 3, EulerCurvFP64>;
    __shared__ double lds[L::LDS_D];
    __shared__ double sref[L::REF_D];
    const auto A = kernel_args<CurvArgs<N>>();
    sf_block<N, 3, EulerCurvFP64>(A->u, A->out, A->E, (int64_t)blockIdx.x * Geom<N, 3>::EPB, KernargOp<N>{&A->op},
                                  A->gamma, lds, sref, VolumeWork{}, A->Ja);
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
    for (int i = 0; i < N * N; ++i) a.op.Q[i] = r.op.Q[i];
    for (int i = 0; i < N; ++i) a.op.w[i] = r.op.w[i];
    hipLaunchKernelGGL((sf_curv_kernel<N>), dim3((unsigned)blocks), dim3(G::THREADS), 0, r.stream, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("sf_curv_kernel launch: ") + hipGetErrorString(err));
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

// ---------------------------------------------------------------------------
// Serving: a batch of requests of mixed n and precision (3D Euler) runs as
// one persistent kernel per (precision, n) variant.  Within a variant, global
// block b belongs to the last request whose blk_begin <= b (a uniform binary
// search) and runs exactly the code of the standalone kernel (sf_block), so
// a request's result does not depend on the batch it is served in.  Blocks
// are visited b = blockIdx.x, + gridDim.x, ... .
// ---------------------------------------------------------------------------
constexpr int serve_table_size(int n) { return n < 2 ? 0 : serve_table_size(n - 1) + n * n + n; }
constexpr int kServeKindDoubles = serve_table_size(kServeMaxN) - serve_table_size(1);
// offset of Q for (node_kind, n) in the table; w follows Q
__host__ __device__ constexpr int serve_table_off(int kind, int n) {
    return kind * kServeKindDoubles + serve_table_size(n - 1);
}

template <int N, class P>
__global__ void __launch_bounds__(kServeThreads, 3)
serve_kernel(const ServeDesc *__restrict__ desc, const int *__restrict__ hdr, const double *__restrict__ optab) {
    static_assert(Geom<N, 3>::THREADS == kServeThreads, "serving assumes 192-thread blocks");
    using L = SfLayout<N, 3, P>;
    __shared__ double lds[L::LDS_D];
    __shared__ double sref[L::REF_D];
    const int ndesc = hdr[0];
    const int total = hdr[1];
    desc += hdr[2];
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        int lo = 0, hi = ndesc - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (desc[mid].blk_begin <= b) lo = mid; else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);  // uniform: keep the descriptor scalar
        const ServeDesc D = desc[lo];
        const int off = __builtin_amdgcn_readfirstlane(serve_table_off(D.node_kind, N));
        const TableOp op{optab + off, optab + off + N * N};
        // gamma is uniform per descriptor: keep it (and the flux constants
        // derived from it) in scalar registers
        const int64_t gbits = __builtin_bit_cast(int64_t, D.gamma);
        const int glo = __builtin_amdgcn_readfirstlane((int)(gbits & 0xffffffff));
        const int ghi = __builtin_amdgcn_readfirstlane((int)(gbits >> 32));
        const double gamma = __builtin_bit_cast(double, ((int64_t)ghi << 32) | (uint32_t)glo);
        sf_block<N, 3, P>(D.u, D.out, D.E, (b - D.blk_begin) * Geom<N, 3>::EPB, op, gamma, lds, sref);
        __syncthreads();  // the next block reuses the LDS
    }
}

}  // namespace dev

int64_t serve_blocks(int n, int64_t E) {
    int epb = 1;
    switch (n) {
        case 2: epb = dev::Geom<2, 3>::EPB; break;
        case 3: epb = dev::Geom<3, 3>::EPB; break;
        case 4: epb = dev::Geom<4, 3>::EPB; break;
        case 5: epb = dev::Geom<5, 3>::EPB; break;
        case 6: epb = dev::Geom<6, 3>::EPB; break;
        case 7: epb = dev::Geom<7, 3>::EPB; break;
        case 8: epb = dev::Geom<8, 3>::EPB; break;
        default: return -1;
    }
    return (E + epb - 1) / epb;
}

int serve_optable_doubles() { return 2 * dev::kServeKindDoubles; }

void serve_fill_optable(double *host) {
    for (int kind = 0; kind < 2; ++kind)
        for (int n = 2; n <= kServeMaxN; ++n) {
            Operator1D op;
            get_operator(n, kind, op);
            double *q = host + dev::serve_table_off(kind, n);
            for (int i = 0; i < n * n; ++i) q[i] = op.Q[i];
            for (int i = 0; i < n; ++i) q[n * n + i] = op.w[i];
        }
}

const void *serve_variant_kernel(int variant) {
    using namespace dev;
    switch (variant) {
        case 0: return reinterpret_cast<const void *>(&serve_kernel<2, EulerFP64>);
        case 1: return reinterpret_cast<const void *>(&serve_kernel<3, EulerFP64>);
        case 2: return reinterpret_cast<const void *>(&serve_kernel<4, EulerFP64>);
        case 3: return reinterpret_cast<const void *>(&serve_kernel<5, EulerFP64>);
        case 4: return reinterpret_cast<const void *>(&serve_kernel<6, EulerFP64>);
        case 5: return reinterpret_cast<const void *>(&serve_kernel<7, EulerFP64>);
        case 6: return reinterpret_cast<const void *>(&serve_kernel<8, EulerFP64>);
        case 7: return reinterpret_cast<const void *>(&serve_kernel<2, EulerFP32Split>);
        case 8: return reinterpret_cast<const void *>(&serve_kernel<3, EulerFP32Split>);
        case 9: return reinterpret_cast<const void *>(&serve_kernel<4, EulerFP32Split>);
        case 10: return reinterpret_cast<const void *>(&serve_kernel<5, EulerFP32Split>);
        case 11: return reinterpret_cast<const void *>(&serve_kernel<6, EulerFP32Split>);
        case 12: return reinterpret_cast<const void *>(&serve_kernel<7, EulerFP32Split>);
        case 13: return reinterpret_cast<const void *>(&serve_kernel<8, EulerFP32Split>);
        default: return nullptr;
    }
}

int launch_sf_volume(const VolumeRequest &r) {
    using namespace dev;
    if (r.precision == SF_PREC_FP32_SPLIT) {
        if (r.flux == SF_FLUX_EULER_CHANDRASHEKAR && r.d == 3)
            return dispatch_n<3, EulerFP32Split, SF_MAX_N_EULER>(r);
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
        default: break;
    }
    set_error("flux / dimension combination not built");
    return SF_ERR_UNSUPPORTED;
}

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
        default: break;
    }
    set_error("flux / dimension combination not built");
    return SF_ERR_UNSUPPORTED;
}

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
