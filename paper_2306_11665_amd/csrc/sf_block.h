// The block-level machinery shared by the sum-factorized kernels (Eq. (3)
// with the coefficients of Eq. (5)): the LDS layout, the operator views and
// sf_block, which runs a block of elements through the steps below with a
// per-line work policy (the volume pairs, the surface term, or both).
//
// One workgroup per block of EPB elements, one line per lane.  Grouped
// mapping (FE = 0): d groups of LPD lanes, group m handling every line of
// direction m of the block's elements (at n = 8 in 3D: one element, 3 waves
// of 64 lanes, 64 lines each; FE < 0: the same over -FE elements per
// block).  Flat mapping (FE > 0 elements per block):
// the lines of all directions laid out one after the other over the lanes,
// the direction a per-lane value (Geom).
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
#pragma once

#include "kernels_common.h"
#include "sfhad_internal.h"

namespace sfhad {
namespace dev {

// Q[i] in the line sums' type (the FP32 copy for FP32 sums: a scalar load,
// no per-lane conversion).
template <class R, class Op>
__device__ __forceinline__ R op_q(const Op &op, int i) {
    if constexpr (sizeof(R) == 4)
        return op.qf(i);
    else
        return op.q(i);
}

// a2..a5 for one line: every unordered pair (a < c) once plus the diagonal,
// accumulated into t.  The loads of the stored arrays are rotated into the
// frame of direction M (a constant after inlining in the grouped mapping, a
// per-lane value in the flat one).  With AHEAD (the standalone volume kernel
// where its launch shape asks for it) the next partner's loads are issued
// before the current pair's arithmetic, so their LDS latency overlaps it.
template <int N, class P, bool AHEAD, class Op>
__device__ __forceinline__ void line_pairs(const int M, const typename P::Real *le, int AS, int pbase, int pstride,
                                           const Op &op, const typename P::Consts &K, double gamma,
                                           typename P::Real (&t)[N][P::NV]) {
    using R = typename P::Real;
    using Node = typename P::Node;
    // node k of the line sits at byte offset pb + k * ps from le; the offset
    // is made opaque at each use, so the compiler re-reads the node from LDS
    // instead of keeping the whole line live in registers
    const int pb = pbase * (int)sizeof(R), ps = pstride * (int)sizeof(R);
    auto at = [&](int k) {
        return reinterpret_cast<const R *>(reinterpret_cast<const char *>(le) + pin(pb + k * ps));
    };
#pragma unroll
    for (int a = 0; a < N; ++a) {
        const Node A = P::load(at(a), AS, 0, M);
        R F[P::NV];
        P::diag(A, gamma, F);
        const R qaa = op_q<R>(op, a * N + a);
#pragma unroll
        for (int k = 0; k < P::NV; ++k) t[a][k] = qaa * F[k] + t[a][k];
        Node C;
        if (AHEAD && a + 1 < N) C = P::load_partner(at(a + 1), AS, 0, M);
#pragma unroll
        for (int c = a + 1; c < N; ++c) {
            Node Cn;
            if (!AHEAD) C = P::load_partner(at(c), AS, 0, M);
            else if (c + 1 < N) Cn = P::load_partner(at(c + 1), AS, 0, M);
            P::pair(A, C, K, F);
            const R qac = op_q<R>(op, a * N + c), qca = op_q<R>(op, c * N + a);
#pragma unroll
            for (int k = 0; k < P::NV; ++k) {
                t[a][k] = qac * F[k] + t[a][k];
                t[c][k] = qca * F[k] + t[c][k];
            }
            // one pair's arithmetic in flight at a time: its sums complete
            // here, before the loads ordered after this fence are issued
#pragma unroll
            for (int k = 0; k < P::NV; ++k) {
                t[a][k] = pin(t[a][k]);
                t[c][k] = pin(t[c][k]);
            }
            if (AHEAD && c + 1 < N) C = Cn;
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
template <int N, int DIM, class P, int FE = 0>
struct SfLayout {
    using G = Geom<N, DIM, FE>;
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
    __device__ float qf(int i) const { return a->Qf[i]; }
    __device__ double w(int i) const { return a->w[i]; }
};

// The same through a reference to the by-value parameter: for the small
// argument blocks (n <= 9) clang keeps it in the argument segment, and the
// kernels come out slightly faster this way.
template <int N>
struct ParamOp {
    const OpArg<N> &a;
    __device__ double q(int i) const { return a.Q[i]; }
    __device__ float qf(int i) const { return a.Qf[i]; }
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
    __device__ float qf(int i) const { return (float)q(i); }
    __device__ double w(int i) const { return W[i]; }
};

// The per-line work of a block.  VolumeWorkT is a2..a5 (every pair of the
// line); SurfaceWork (with the surface kernels) is the facet part of the
// surface term, and with VOLUME it adds the pairs into the same line sums.
template <bool AHEAD>
struct VolumeWorkT {
    template <int M, int N, class P, class Op, class R>
    __device__ __forceinline__ void lines(const R *le, int AS, int pbase, int pstride, const Op &op,
                                          const typename P::Consts &K, double gamma, R (&t)[N][P::NV], int64_t,
                                          int, double, const double *) const {
        line_pairs<N, P, AHEAD>(M, le, AS, pbase, pstride, op, K, gamma, t);
    }
    // the same with the direction a per-lane value (flat mapping)
    template <int N, class P, class Op, class R>
    __device__ __forceinline__ void lines_rt(int m, const R *le, int AS, int pbase, int pstride, const Op &op,
                                             const typename P::Consts &K, double gamma, R (&t)[N][P::NV]) const {
        line_pairs<N, P, AHEAD>(m, le, AS, pbase, pstride, op, K, gamma, t);
    }
};
using VolumeWork = VolumeWorkT<false>;  // serving and curvilinear kernels (register-capped)

// One block of EPB elements starting at element e0 of an E-element mesh:
// steps a1..a6 with the line work of `work`.  lds holds SfLayout::LDS_D
// doubles, sref SfLayout::REF_D.  FE selects the lane mapping (Geom); the
// flat mapping is built for the volume pairs only.
template <int N, int DIM, class P, int FE = 0, bool OWNREF = false, class Op, class Work = VolumeWork>
__device__ __forceinline__ void sf_block(const double *__restrict__ u, double *__restrict__ out, int64_t E,
                                         int64_t e0, const Op &op, double gamma, double *lds, double *sref,
                                         const Work &work = Work{}, const double *__restrict__ aux = nullptr) {
    using G = Geom<N, DIM, FE>;
    using L = SfLayout<N, DIM, P, FE>;
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

    // a1: every load of the staging pass is issued before any conversion
    // (one memory round trip for the whole stage)
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
    // OWNREF with one element per block: every thread derives the element's
    // reference values itself from the element's first node (one address
    // for all lanes), so the stage needs no barrier of its own (the
    // standalone volume kernel: 1.03x at n = 8; the registers it keeps live
    // make the surface and serving kernels spill, so they do not take it).
    // Otherwise the thread holding an element's first node derives them into
    // LDS, then a barrier.
    constexpr bool kOwnRef = OWNREF && G::EPB == 1 && P::NREF > 0;
    double rloc[NREF];
    if constexpr (kOwnRef) {
        double u0[P::NV + P::NX];
#pragma unroll
        for (int v = 0; v < P::NV; ++v) u0[v] = u[v * vstride + gbase];
#pragma unroll
        for (int x = 0; x < P::NX; ++x) u0[P::NV + x] = aux[x * vstride + gbase];
        P::make_ref(u0, gamma, rloc);
        if (tid == 0) {
#pragma unroll
            for (int q = 0; q < NREF; ++q) sref[q] = rloc[q];  // for the line work, after the next barrier
        }
    } else if (P::NREF > 0) {
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int i = tid + k * G::THREADS;
            if (i < nvalid && i % G::NODES == 0) P::make_ref(uc[k], gamma, sref + (i / G::NODES) * NREF);
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int i = tid + k * G::THREADS;
        if (i < nvalid) {
            R s[P::NS];
            P::stage(uc[k], kOwnRef ? rloc : sref + (i / G::NODES) * NREF, gamma, s);
            const int el = i / G::NODES, node = i - el * G::NODES;
            const int li = el * G::PADN + G::pidx(node);
#pragma unroll
            for (int q = 0; q < P::NS; ++q) lin[q * AS + li] = s[q];
        }
    }
    __syncthreads();

    // a2..a5: one line per lane.
    int el, m, line;
    G::lane(tid, el, m, line);
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

    if constexpr (FE > 0) {
        // the direction varies across the wave: one instantiation with
        // per-lane array offsets
        if (active) work.template lines_rt<N, P>(m, le, AS, pbase, pstride, op, K, gamma, t);
    } else if (active) {
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
    // direction cover consecutive nodes: coalesced).  In the flat mapping a
    // wave may hold lanes of several directions; each lane takes part in
    // the round of its own direction.
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

}  // namespace dev
}  // namespace sfhad
