// Serving kernels of the volume term (Eq. (3) with the coefficients of
// Eq. (5)) for batches of requests of mixed n and precision, and the host
// helpers the serving runtime uses to size and launch them.
#include "sf_block.h"

namespace sfhad {
namespace dev {

// ---------------------------------------------------------------------------
// Serving: a batch of requests of mixed n and precision (3D Euler) runs as
// one kernel launch per (precision, n) variant, one workgroup per block of
// elements.  Within a variant, global block b belongs to the last request
// whose blk_begin <= b (a uniform binary search) and runs exactly the code
// of the standalone kernel (sf_block), so a request's result does not depend
// on the batch it is served in.
// ---------------------------------------------------------------------------
constexpr int serve_table_size(int n) { return n < 2 ? 0 : serve_table_size(n - 1) + n * n + n; }
constexpr int kServeKindDoubles = serve_table_size(kServeMaxN) - serve_table_size(1);
// offset of Q for (node_kind, n) in the table; w follows Q
__host__ __device__ constexpr int serve_table_off(int kind, int n) {
    return kind * kServeKindDoubles + serve_table_size(n - 1);
}

// The serving kernels take the standalone kernel's lane mapping (flat where
// it fills more lanes) and look-ahead choice, at least 3 waves per SIMD.
template <int N, class P>
constexpr int serve_fe() {
    return euler_volume_shape(N, sizeof(typename P::Real) == 8).fe;
}
template <int N, class P>
constexpr bool serve_ahead() {
    return euler_volume_shape(N, sizeof(typename P::Real) == 8).ahead;
}

template <int N, class P>
__global__ void __launch_bounds__((Geom<N, 3, serve_fe<N, P>()>::THREADS), 3)
serve_kernel(const ServeArgs) {
    constexpr int FE = serve_fe<N, P>();
    using L = SfLayout<N, 3, P, FE>;
    __shared__ double lds[L::LDS_D];
    __shared__ double sref[L::REF_D];
    const auto A = kernel_args<ServeArgs>();
    // the descriptors: a device array, or the argument block itself (the
    // kernel-argument segment is ordinary readable memory); global address
    // space, so that the uniform reads stay scalar loads
    using GDesc = const __attribute__((address_space(1))) ServeDesc;
    GDesc *__restrict__ dd = A->desc ? (GDesc *)A->desc : (GDesc *)&A->inl[0];
    const int ndesc = A->ndesc;
    // one workgroup per block of elements (a grid-stride loop over the
    // blocks kept the loop's state live through the pair phase: 16-96 bytes
    // of spills per lane and 0.86 of this form's burst throughput)
    const int b = blockIdx.x;
    if (b >= A->total) return;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (dd[mid].blk_begin <= b) lo = mid; else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);  // uniform: keep the descriptor scalar
    GDesc &D = dd[lo];
    const int off = __builtin_amdgcn_readfirstlane(serve_table_off(D.node_kind, N));
    const TableOp op{A->optab + off, A->optab + off + N * N};
    // gamma is uniform per descriptor: keep it (and the flux constants
    // derived from it) in scalar registers
    const int64_t gbits = __builtin_bit_cast(int64_t, D.gamma);
    const int glo = __builtin_amdgcn_readfirstlane((int)(gbits & 0xffffffff));
    const int ghi = __builtin_amdgcn_readfirstlane((int)(gbits >> 32));
    const double gamma = __builtin_bit_cast(double, ((int64_t)ghi << 32) | (uint32_t)glo);
    sf_block<N, 3, P, FE>(D.u, D.out, D.E, (b - D.blk_begin) * Geom<N, 3, FE>::EPB, op, gamma, lds, sref,
                          VolumeWorkT<serve_ahead<N, P>()>{});
}

}  // namespace dev

namespace {
template <int N>
void serve_geom(int prec, int &epb, int &threads) {
    if (prec == SF_PREC_FP32_SPLIT) {
        using G = dev::Geom<N, 3, dev::serve_fe<N, dev::EulerFP32Split>()>;
        epb = G::EPB;
        threads = G::THREADS;
    } else {
        using G = dev::Geom<N, 3, dev::serve_fe<N, dev::EulerFP64>()>;
        epb = G::EPB;
        threads = G::THREADS;
    }
}

bool serve_geom(int n, int prec, int &epb, int &threads) {
    switch (n) {
        case 2: serve_geom<2>(prec, epb, threads); return true;
        case 3: serve_geom<3>(prec, epb, threads); return true;
        case 4: serve_geom<4>(prec, epb, threads); return true;
        case 5: serve_geom<5>(prec, epb, threads); return true;
        case 6: serve_geom<6>(prec, epb, threads); return true;
        case 7: serve_geom<7>(prec, epb, threads); return true;
        case 8: serve_geom<8>(prec, epb, threads); return true;
        default: return false;
    }
}
}  // namespace

int64_t serve_blocks(int n, int prec, int64_t E) {
    int epb, threads;
    if (!serve_geom(n, prec, epb, threads)) return -1;
    return (E + epb - 1) / epb;
}

int serve_threads(int variant) {
    int epb = 1, threads = 0;
    serve_geom(variant % (kServeMaxN - 1) + 2, variant / (kServeMaxN - 1), epb, threads);
    return threads;
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

}  // namespace sfhad
