// Sum-factorized basis transformation (the step the proof of Theorem 1 adds
// in front of the Hadamard product): out_e = (M (x) ... (x) M) in_e for every
// element and variable, applied as d one-dimensional passes (Eq. (6): the
// modal basis chi evaluated on the nodes, M = V, or its projection, M = P).
//
// Each pass is a small dense contraction: for direction m, every grid line L
// of a slab (one element's values of one variable, n^d doubles) maps
// Y_L[q] = sum_k M[q][k] X_L[k].  It runs on the FP64 matrix cores:
// v_mfma_f64_16x16x4f64 computes D(16 x 16) += A(16 x 4) B(4 x 16) with
//   A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
//   D[i][j] in lane j + 16 (i % 4), accumulator register i / 4
// (the layout verified on gfx950).  Here i = output node q (n <= 16 of the
// 16 rows used), j = one of 16 lines, k = input node, ceil(n / 4) steps.
//
// The work is HBM-bound (2 x 8 bytes per value moved against 2 d n flops),
// so a block streams G slabs (at most 2048 values and 256 lines) through one
// LDS buffer: coalesced loads of all its slabs, d - 1 passes that keep their
// (at most 4) tiles in registers and overwrite the buffer after a barrier,
// and the last pass written from the MFMA accumulators straight to HBM (for
// the last direction the 16 lines of a tile are 16 consecutive nodes:
// 128-byte segments).  One buffer instead of two doubles the blocks, and so
// the loads in flight, per CU.  A block only writes the slabs it read, after
// a barrier, so in == out is allowed.
#include "kernels_common.h"
#include "entropy_maps.h"
#include "tensor_internal.h"

namespace sfhad {
namespace dev {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTensorThreads = 256;

template <int N>
struct MatArg {
    double M[N * N];
};

template <int N, int DIM>
struct TensorGeom {
    static constexpr int NODES = DIM == 3 ? N * N * N : N * N;
    static constexpr int LINES = NODES / N;                          // lines per slab and direction
    static constexpr int GV = NODES >= 2048 ? 1 : 2048 / NODES;      // by values per block
    static constexpr int GL = LINES >= 256 ? 1 : 256 / LINES;        // by lines per block
    static constexpr int G = GV < GL ? GV : GL;                      // slabs per block
    static constexpr int PADN = NODES + LINES;                       // one pad slot per x-row
    static constexpr int KS = (N + 3) / 4;                           // MFMA k-steps
    static constexpr int TILES = (G * LINES + 15) / 16;              // 16-line tiles per pass
    static constexpr int TPW = (TILES + 3) / 4;                      // tiles per wave (<= 4)
};

// padded LDS index of node `nd` of slab g
template <int N, int DIM>
__device__ __forceinline__ int tpad(int g, int nd) {
    return g * TensorGeom<N, DIM>::PADN + nd + nd / N;
}

// node of line L, position k, in direction m (x fastest)
template <int N, int DIM>
__device__ __forceinline__ int tnode(int L, int k, int m) {
    if (DIM == 2) return m == 0 ? k + N * L : L + N * k;
    if (m == 0) return k + N * L;                         // L = y + n z
    if (m == 1) return (L % N) + N * k + N * N * (L / N);  // L = x + n z
    return L + N * N * k;                                 // L = x + n y
}

template <int N, int DIM>
__global__ void __launch_bounds__(kTensorThreads)
tensor_apply_kernel(const double *__restrict__ in, double *out, int64_t slabs, MatArg<N> M) {
    using G = TensorGeom<N, DIM>;
    static_assert(G::TPW <= 4, "at most 4 tiles per wave are held in registers");
    __shared__ double buf[G::G * G::PADN];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * G::G;
    const int gs = (int)((slabs - s0) < G::G ? (slabs - s0) : G::G);  // slabs in this block
    const int nvals = gs * G::NODES;
    const double *src = in + s0 * G::NODES;

    // coalesced load of the block's slabs (every load issued before any store)
    constexpr int PER = (G::G * G::NODES + kTensorThreads - 1) / kTensorThreads;
    double v[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = tid + j * kTensorThreads;
        v[j] = i < nvals ? src[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int i = tid + j * kTensorThreads;
        if (i < nvals) buf[tpad<N, DIM>(i / G::NODES, i % G::NODES)] = v[j];
    }

    // A operand per k-step: M[q][k], q = lane % 16, k = 4 s + lane / 16
    double a[G::KS];
    const int q_a = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int s = 0; s < G::KS; ++s) {
        const int k = 4 * s + kq;
        a[s] = (q_a < N && k < N) ? M.M[q_a * N + k] : 0.0;
    }
    __syncthreads();

    const int nlines = gs * G::LINES;
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        d4 acc[G::TPW];
#pragma unroll
        for (int u = 0; u < G::TPW; ++u) {
            const int t = wave + 4 * u;  // wave-uniform: every lane runs the MFMA
            acc[u] = d4{0.0, 0.0, 0.0, 0.0};
            if (t >= G::TILES) continue;
            const int Lg = t * 16 + (lane & 15);  // this lane's line (B column, D column)
            const bool lok = Lg < nlines;
            const int g = lok ? Lg / G::LINES : 0;
            const int L = lok ? Lg % G::LINES : 0;
#pragma unroll
            for (int s = 0; s < G::KS; ++s) {
                const int k = 4 * s + kq;
                const double b = (lok && k < N) ? buf[tpad<N, DIM>(g, tnode<N, DIM>(L, k, m))] : 0.0;
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b, acc[u], 0, 0, 0);
            }
        }
        if (m < DIM - 1) __syncthreads();  // every read of this pass is done
        // D[q][line] in register r, q = 4 r + lane / 16
#pragma unroll
        for (int u = 0; u < G::TPW; ++u) {
            const int t = wave + 4 * u;
            if (t >= G::TILES) continue;
            const int Lg = t * 16 + (lane & 15);
            if (Lg >= nlines) continue;
            const int g = Lg / G::LINES;
            const int L = Lg % G::LINES;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = 4 * r + kq;
                if (q >= N) continue;
                const int nd = tnode<N, DIM>(L, q, m);
                if (m == DIM - 1)
                    out[(s0 + g) * G::NODES + nd] = acc[u][r];
                else
                    buf[tpad<N, DIM>(g, nd)] = acc[u][r];
            }
        }
        if (m < DIM - 1) __syncthreads();  // the pass's results are in place
    }
}

template <int N, int DIM>
int launch_tensor(const TensorRequest &r) {
    using G = TensorGeom<N, DIM>;
    MatArg<N> M;
    for (int i = 0; i < N * N; ++i) M.M[i] = r.M[i];
    const int64_t slabs = r.E * r.nvar;
    const int64_t blocks = (slabs + G::G - 1) / G::G;
    if (blocks > 0x7fffffffLL) {
        set_error("too many elements for one launch");
        return SF_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL((tensor_apply_kernel<N, DIM>), dim3((unsigned)blocks), dim3(kTensorThreads), 0, r.stream,
                       r.in, r.out, slabs, M);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        set_error(std::string("tensor_apply_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

template <int DIM>
int dispatch_tensor(const TensorRequest &r) {
    switch (r.n) {
        case 2: return launch_tensor<2, DIM>(r);
        case 3: return launch_tensor<3, DIM>(r);
        case 4: return launch_tensor<4, DIM>(r);
        case 5: return launch_tensor<5, DIM>(r);
        case 6: return launch_tensor<6, DIM>(r);
        case 7: return launch_tensor<7, DIM>(r);
        case 8: return launch_tensor<8, DIM>(r);
        case 9: return launch_tensor<9, DIM>(r);
        case 10: return launch_tensor<10, DIM>(r);
        case 11: return launch_tensor<11, DIM>(r);
        case 12: return launch_tensor<12, DIM>(r);
        case 13: return launch_tensor<13, DIM>(r);
        case 14: return launch_tensor<14, DIM>(r);
        case 15: return launch_tensor<15, DIM>(r);
        case 16: return launch_tensor<16, DIM>(r);
        default:
            set_error("n outside [2, 16]");
            return SF_ERR_UNSUPPORTED;
    }
}

// ---------------------------------------------------------------------------
// Rectangular form: M is n_out x n_in (n modes to m quadrature nodes or
// back), sizes at run time (2 <= n_in, n_out <= 16).  Pass m turns extent
// n_in into n_out along direction m, so the intermediate stages have mixed
// extents (directions before m already n_out); each stage is stored with x
// fastest and one pad slot per x-row.  Same MFMA scheme and in-place single
// buffer as the square kernel; the A operand rows q < n_out, k < n_in.
//
// Every index split divides by a run-time size (n_in, n_out, n_in^d, the
// lines per slab of a pass).  Instead of integer division (a long
// instruction sequence) the kernel multiplies by a reciprocal from the host:
// floor(x / d) = mulhi(x, ceil(2^32 / d)) exactly when x e < 2^32,
// e = ceil(2^32 / d) d - 2^32 < d (write x = q d + r: the product is
// q + r/d + x e / (d 2^32), below q + 1 when r <= d - 1 and x e < 2^32).
// Here d <= 4352 and x <= 4352 (an index inside the block's LDS stage of
// at most kRectStage values plus pads, or its lines), so x e < 2^25.
constexpr int kRectTPW = 8;       // 16-line tiles per wave and pass (at most)
constexpr int kRectStage = 4096;  // LDS doubles per block for the slabs (plus pads), run-time sizes
// The same for the compile-time size pairs, from A/B runs on MI355X against
// 4096: 6144 (more slabs per block) ran 1.03-1.17x faster for every pair
// measured (3 -> 5 up to 9 -> 7) but the projection from 10^3 nodes, which
// ran faster with fewer (3072: 1.07x at 10 -> 8; 6144: 0.93x; 2048: 0.92x
// of 3072).
__host__ __device__ constexpr int rect_stage(int ni, int no) {
    return (ni > no && ni * ni * ni >= 1000) ? 3072 : 6144;
}

struct RectArgs {
    const double *in;
    double *out;
    int64_t slabs;
    double gamma;  // the fused pointwise map's (MAP != 0)
    int ni, no, G, cap;  // sizes, slabs per block, LDS doubles per slab
    uint32_t rc_ni, rc_no, rc_nin;  // ceil(2^32 / d) of n_in, n_out, n_in^d
    uint32_t rc_lps[3];             // of the lines per slab of pass m
    double M[kMaxN * kMaxN];  // row-major n_out x n_in (row stride n_in)
};

__device__ __forceinline__ int qdiv(int x, uint32_t rc) { return (int)__umulhi((uint32_t)x, rc); }
// index products: every factor is below 2^16, so the full-rate 24-bit multiply is exact
__device__ __forceinline__ int m24(int a, int b) { return __mul24(a, b); }

__host__ __device__ constexpr uint32_t rect_rc(int64_t d) {
    return (uint32_t)(((int64_t)1 << 32) / d + ((((int64_t)1 << 32) % d) != 0));
}
__host__ __device__ constexpr int rect_pow(int b, int e) { return e == 0 ? 1 : b * rect_pow(b, e - 1); }
// slabs per block: the LDS stage holds `stage` doubles, and the lines of a
// pass fill at most 4 waves x kRectTPW tiles of 16
__host__ __device__ constexpr int rect_slabs_per_block(int ni, int no, int d, int stage) {
    const int mx = ni > no ? ni : no;
    const int mxd = rect_pow(mx, d), mxl = rect_pow(mx, d - 1);
    const int g1 = stage / mxd, g2 = 64 * kRectTPW / mxl;
    const int g = g1 < g2 ? g1 : g2;
    return g < 1 ? 1 : g;
}

// Slabs per block of the fused form: the 5 variables of whole elements.
__host__ __device__ constexpr int rect_map_slabs_per_block(int ni, int no) {
    return rect_slabs_per_block(ni, no, 3, rect_stage(ni, no)) / 5 * 5;
}

// NI, NO > 0: the sizes as compile-time constants (every index split and
// product folds into shifts and constant multiplies); 0: run-time sizes
// from the arguments.  The code is the same.  MAP != 0 (3D Euler, 5
// variables, n_out = n_in + 2 or n_out = n_in): a block takes the 5 variable
// slabs of whole elements, keeps the last pass in LDS and applies a
// pointwise map to each output node before the store -- conserved to
// entropy variables (MAP = 1) or back (MAP = 2) -- so the map costs no
// separate pass over HBM.
template <int DIM, int NI, int NO, int MAP = 0>
__global__ void __launch_bounds__(kTensorThreads) tensor_rect_kernel(const RectArgs) {
    extern __shared__ double buf[];
    const auto A = kernel_args<RectArgs>();
    constexpr bool CT = NI > 0 && NO > 0;
    static_assert(MAP == 0 || (CT && DIM == 3 && NI <= NO), "the fused map is built for 3D, n_out >= n_in");
    constexpr int MX = NI > NO ? NI : NO;
    const int ni = CT ? NI : A->ni, no = CT ? NO : A->no;
    constexpr int STAGE = CT ? rect_stage(NI, NO) : kRectStage;
    const int G = MAP ? rect_map_slabs_per_block(NI, NO) : (CT ? rect_slabs_per_block(NI, NO, DIM, STAGE) : A->G);
    const int cap = CT ? rect_pow(MX, DIM) + rect_pow(MX, DIM - 1) : A->cap;
    const uint32_t rc_ni = CT ? rect_rc(NI) : A->rc_ni, rc_no = CT ? rect_rc(NO) : A->rc_no;
    const uint32_t rc_nin = CT ? rect_rc(rect_pow(NI, DIM)) : A->rc_nin;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int nin = 1, nout = 1;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        nin *= ni;
        nout *= no;
    }
    // slabs of this block: s0 .. s0 + gs - 1; with MAP, element-major over the
    // block's elements e0 .. e0 + gs/5 - 1 (block slab g = 5 el + var is the
    // global slab var * E + e0 + el)
    const int64_t E5 = A->slabs / 5;
    const int64_t s0 = (int64_t)blockIdx.x * G;
    const int64_t e0 = (int64_t)blockIdx.x * (G / 5);
    const int gs = MAP ? 5 * (int)((E5 - e0) < G / 5 ? (E5 - e0) : G / 5)
                       : (int)((A->slabs - s0) < G ? (A->slabs - s0) : G);
    const double *src = A->in + s0 * nin;
    // stage 0: the input slabs, x fastest, one pad per x-row of n_in; every
    // load is issued before the first LDS store
    constexpr int SPT = STAGE / kTensorThreads;
    const int total = gs * nin;
    double v[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = tid + j * kTensorThreads;
        if (i < total) {
            if constexpr (MAP != 0) {
                const int g = qdiv(i, rc_nin), lin = i - m24(g, nin);
                v[j] = A->in[((int64_t)(g % 5) * E5 + e0 + g / 5) * nin + lin];
            } else {
                v[j] = src[i];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int i = tid + j * kTensorThreads;
        if (i < total) {
            const int g = qdiv(i, rc_nin), lin = i - m24(g, nin);
            buf[m24(g, cap) + lin + qdiv(lin, rc_ni)] = v[j];
        }
    }
    const int q_a = lane & 15, kq = lane >> 4;
    double a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + kq;
        a[s] = (q_a < no && k < ni) ? A->M[q_a * ni + k] : 0.0;
    }
    const int ks = (ni + 3) >> 2;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        // extents at stage m (before the pass) and stage m + 1 (after)
        int ext[3], exo[3];
        uint32_t rce[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ext[k] = k < DIM ? (k < m ? no : ni) : 1;
            exo[k] = k < DIM ? (k <= m ? no : ni) : 1;
            rce[k] = k < m ? rc_no : rc_ni;  // used for k < DIM, k != m only
        }
        int lps = 1;  // lines per slab
#pragma unroll
        for (int k = 0; k < DIM; ++k)
            if (k != m) lps *= ext[k];
        const int nlines = gs * lps;
        const int tiles = (nlines + 15) >> 4;
        // Padded stage index of coordinates c (x fastest, one pad per x-row):
        // c0 + ext0 R + floor((c0 + ext0 R) / ext0) = c0 + (ext0 + 1) R with
        // R = c1 + ext1 c2, so a line of direction m is base + k * stride.
        const int si1 = ext[0] + 1, si2 = (ext[0] + 1) * ext[1];
        const int so1 = exo[0] + 1, so2 = (exo[0] + 1) * exo[1];
        const int sg1 = exo[0], sg2 = exo[0] * exo[1];  // unpadded (the output array)
        const int str_in = m == 0 ? 1 : (m == 1 ? si1 : si2);
        const int str_out = m == 0 ? 1 : (m == 1 ? so1 : so2);
        const int str_g = m == 0 ? 1 : (m == 1 ? sg1 : sg2);
        const bool to_lds = m < DIM - 1 || MAP != 0;  // this pass's results stay in LDS
        d4 acc[kRectTPW];
        int bout[kRectTPW];  // output base: LDS index, or the element offset in `out`
        bool ok[kRectTPW];
#pragma unroll
        for (int u = 0; u < kRectTPW; ++u) {
            const int t = wave + 4 * u;  // wave-uniform
            acc[u] = d4{0.0, 0.0, 0.0, 0.0};
            ok[u] = false;
            bout[u] = 0;
            if (t >= tiles) continue;
            const int Lg = t * 16 + (lane & 15);
            ok[u] = Lg < nlines;
            uint32_t rc_lps = A->rc_lps[m];
            if (CT) {
                int lp = 1;
#pragma unroll
                for (int k = 0; k < DIM; ++k)
                    if (k != m) lp *= k < m ? NO : NI;
                rc_lps = rect_rc(lp);
            }
            const int g = ok[u] ? qdiv(Lg, rc_lps) : 0;
            int L = ok[u] ? Lg - m24(g, lps) : 0;
            // coordinates of the other directions, increasing order, first fastest
            int c[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                if (k == m) continue;
                const int qk = qdiv(L, rce[k]);
                c[k] = L - m24(qk, ext[k]);
                L = qk;
            }
            const int bin = m24(g, cap) + c[0] + m24(si1, c[1]) + m24(si2, c[2]);
            bout[u] = !to_lds ? m24(g, nout) + c[0] + m24(sg1, c[1]) + m24(sg2, c[2])
                              : m24(g, cap) + c[0] + m24(so1, c[1]) + m24(so2, c[2]);
            // the tile's B operands first (up to 4 LDS reads in flight), then
            // the MFMAs; ks is wave-uniform
            double b[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 4 * s + kq;
                b[s] = (s < ks && ok[u] && k < ni) ? buf[bin + m24(k, str_in)] : 0.0;
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if (s < ks) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], acc[u], 0, 0, 0);
        }
        if (to_lds) __syncthreads();  // every read of this pass is done
        double *dst = A->out + s0 * nout;
#pragma unroll
        for (int u = 0; u < kRectTPW; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = 4 * r + kq;
                if (q >= no) continue;
                if (!to_lds)
                    dst[bout[u] + m24(q, str_g)] = acc[u][r];
                else
                    buf[bout[u] + m24(q, str_out)] = acc[u][r];
            }
        }
        if (to_lds) __syncthreads();
    }
    if constexpr (MAP != 0) {
        // the block's output nodes, node fastest (coalesced stores); the last
        // pass left node (x, y, z) of slab g at g cap + node + node / n_out
        const double gam = A->gamma;
        const double igm1 = 1.0 / (gam - 1.0);
        const int nel = gs / 5;
        for (int j = tid; j < nel * nout; j += kTensorThreads) {
            const int el = j / nout, node = j - el * nout;
            const int li = node + node / no;
            double x[5], y[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) x[c] = buf[m24(5 * el + c, cap) + li];
            if (MAP == 1)
                entropy_from_conserved(x, gam, igm1, y);
            else
                conserved_from_entropy(x, gam, igm1, y);
#pragma unroll
            for (int c = 0; c < 5; ++c) A->out[((int64_t)c * E5 + e0 + el) * nout + node] = y[c];
        }
    }
}

}  // namespace dev

int launch_tensor_apply(const TensorRequest &r) {
    if (r.n_out != r.n || r.post_map != SF_MAP_NONE) return launch_tensor_rect(r);
    if (r.d == 2) return dev::dispatch_tensor<2>(r);
    if (r.d == 3) return dev::dispatch_tensor<3>(r);
    set_error("d must be 2 or 3");
    return SF_ERR_UNSUPPORTED;
}

int launch_tensor_rect(const TensorRequest &r) {
    using namespace dev;
    RectArgs a;
    a.in = r.in;
    a.out = r.out;
    a.slabs = r.E * r.nvar;
    a.ni = r.n;
    a.no = r.n_out;
    const int mx = r.n > r.n_out ? r.n : r.n_out;
    a.cap = rect_pow(mx, r.d) + rect_pow(mx, r.d - 1);
    a.rc_ni = rect_rc(r.n);
    a.rc_no = rect_rc(r.n_out);
    a.rc_nin = rect_rc(rect_pow(r.n, r.d));
    for (int m = 0; m < 3; ++m) {
        int lps = 1;
        for (int k = 0; k < r.d; ++k)
            if (k != m) lps *= k < m ? r.n_out : r.n;
        a.rc_lps[m] = m < r.d ? rect_rc(lps) : 0;
    }
    for (int i = 0; i < r.n_out * r.n; ++i) a.M[i] = r.M[i];
    a.gamma = r.gamma;
    // compile-time sizes for the over-integration pairs of the modal path
    // (n modes <-> n + 2 quadrature nodes, n = 3..8, 3D); run-time otherwise
    const void *fn = nullptr;
    if (r.post_map != SF_MAP_NONE) {
        // the fused map: 3D, 5 variables, n -> n + 2 (n = 3..8) or n -> n
        // (n = 3..10, e.g. the projection V P on the quadrature nodes)
        const bool up = r.n_out == r.n + 2 && r.n >= 3 && r.n <= 8, sq = r.n_out == r.n && r.n >= 3 && r.n <= 10;
        if (r.d != 3 || r.nvar != 5 || !(up || sq)) {
            set_error("the fused map is built for 3D Euler states, n -> n + 2 (n = 3..8) or n -> n (n = 3..10)");
            return SF_ERR_UNSUPPORTED;
        }
#define SF_RECT_MAP(NI_, NO_)                                                                              \
        if (r.n == NI_ && r.n_out == NO_)                                                                  \
            fn = r.post_map == SF_MAP_ENTROPY_VARIABLES                                                    \
                     ? reinterpret_cast<const void *>(&tensor_rect_kernel<3, NI_, NO_, SF_MAP_ENTROPY_VARIABLES>) \
                     : reinterpret_cast<const void *>(&tensor_rect_kernel<3, NI_, NO_, SF_MAP_CONSERVED_VARIABLES>);
        SF_RECT_MAP(3, 5) SF_RECT_MAP(4, 6) SF_RECT_MAP(5, 7) SF_RECT_MAP(6, 8) SF_RECT_MAP(7, 9) SF_RECT_MAP(8, 10)
        SF_RECT_MAP(3, 3) SF_RECT_MAP(4, 4) SF_RECT_MAP(5, 5) SF_RECT_MAP(6, 6) SF_RECT_MAP(7, 7) SF_RECT_MAP(8, 8)
        SF_RECT_MAP(9, 9) SF_RECT_MAP(10, 10)
#undef SF_RECT_MAP
        a.G = rect_map_slabs_per_block(r.n, r.n_out);
    } else {
        if (r.d == 3) {
#define SF_RECT(NI_, NO_) \
            if (r.n == NI_ && r.n_out == NO_) fn = reinterpret_cast<const void *>(&tensor_rect_kernel<3, NI_, NO_>);
            SF_RECT(3, 5) SF_RECT(5, 3) SF_RECT(4, 6) SF_RECT(6, 4) SF_RECT(5, 7) SF_RECT(7, 5)
            SF_RECT(6, 8) SF_RECT(8, 6) SF_RECT(7, 9) SF_RECT(9, 7) SF_RECT(8, 10) SF_RECT(10, 8)
#undef SF_RECT
        }
        a.G = rect_slabs_per_block(r.n, r.n_out, r.d, fn ? rect_stage(r.n, r.n_out) : kRectStage);
        if (!fn)
            fn = reinterpret_cast<const void *>(r.d == 3 ? &tensor_rect_kernel<3, 0, 0> : &tensor_rect_kernel<2, 0, 0>);
    }
    const int64_t blocks = r.post_map != SF_MAP_NONE ? (r.E + a.G / 5 - 1) / (a.G / 5) : (a.slabs + a.G - 1) / a.G;
    if (blocks > 0x7fffffffLL) {
        set_error("too many elements for one launch");
        return SF_ERR_UNSUPPORTED;
    }
    const size_t lds = sizeof(double) * (size_t)a.G * a.cap;
    void *kp[] = {&a};
    if (hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(kTensorThreads), kp, lds, r.stream) != hipSuccess) {
        set_error(std::string("tensor_rect_kernel launch: ") + hipGetErrorString(hipGetLastError()));
        return SF_ERR_HIP;
    }
    return SF_OK;
}

}  // namespace sfhad
