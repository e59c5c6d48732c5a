// Device-side building blocks shared by the volume kernels: element/line
// geometry, the LDS layout, and the two-point flux policies.
//
// Geometry.  A line in direction m is the set of n nodes that differ only in
// their index along m (the node pairs Algorithm 1 enumerates); an element
// has n^(d-1) lines per direction.  The kernels give every line to one lane,
// so the coefficient of the pair (a, c) on a line is Q[a][c] times the
// weights of the two (or one) other indices, which are constant along the
// line (Algorithm 2's Basis_Sparse values): w_perp is applied once per line
// after the reduction.
//
// LDS layout.  Per element, each stored per-node quantity is an array of n^d
// doubles with one pad slot after every n nodes (padded index
// node + node / n), which spreads the three line strides (1, n, n^2) of a
// wave's 64 lanes over distinct banks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sfhad {
namespace dev {

// Copy of the 1D operator for a compile-time n, passed by value in the
// kernel arguments (read through the scalar cache: every lane of a wave
// uses the same Q[a][c] at the same time).
template <int N>
struct OpArg {
    double Q[N * N];
    double w[N];
    float Qf[N * N];  // Q rounded to FP32, for the FP32-split form's line sums
};

// Fill an OpArg from a host operator (op.Q, op.w of n = N).
template <int N, class Op1D>
void fill_op_arg(OpArg<N> &a, const Op1D &op) {
    for (int i = 0; i < N * N; ++i) {
        a.Q[i] = op.Q[i];
        a.Qf[i] = (float)op.Q[i];
    }
    for (int i = 0; i < N; ++i) a.w[i] = op.w[i];
}

// The whole argument block of a standalone volume kernel, its only
// parameter.  Kernels read it through the kernel-argument segment pointer
// (constant address space, so the reads are scalar loads): naming the
// by-value parameter directly makes clang copy it into private memory, and
// once the block is too large to split into registers (n >= 11) every
// operator read would be a scratch access.
template <int N>
struct VolArgs {
    const double *u;
    double *out;
    int64_t E;
    double gamma;
    OpArg<N> op;
};

template <class T>
using kernarg_ptr = const __attribute__((address_space(4))) T *;

// The argument block of the running kernel (its first and only parameter
// starts at offset 0 of the segment).
template <class T>
__device__ __forceinline__ kernarg_ptr<T> kernel_args() {
    return (kernarg_ptr<T>)__builtin_amdgcn_kernarg_segment_ptr();
}

// Lane mapping of a block.  FE = 0 ("grouped"): d groups of LPD lanes,
// group m taking every line of direction m of the block's EPB elements, so
// that each wave works on one direction.  FE > 0 ("flat"): FE elements per
// block and their d n^(d-1) lines of every direction laid out one after the
// other over the block's lanes (element, then direction, then line), so
// that a wave may hold lines of several directions; the flux code then
// takes the direction as a per-lane value.  The flat mapping fills the
// lanes when n^(d-1) does not divide into 64 (n = 6, 9, 12, ...).  FE < 0:
// the grouped mapping over -FE elements per block (each direction group
// takes the lines of all of them, the group rounded up to whole waves).
template <int N, int DIM, int FE = 0>
struct Geom {
    static constexpr int LINES = DIM == 3 ? N * N : N;       // lines per direction per element
    static constexpr int NODES = LINES * N;                  // n^d
    static constexpr int EPB = FE > 0 ? FE : FE < 0 ? -FE : (LINES >= 64 ? 1 : 64 / LINES);  // elements per block
    static constexpr int LPD = ((EPB * LINES + 63) / 64) * 64;  // lanes per direction group (grouped)
    static constexpr int LANES = FE > 0 ? EPB * DIM * LINES : DIM * LPD;  // lanes with a line (flat: all)
    static constexpr int THREADS = FE > 0 ? ((LANES + 63) / 64) * 64 : DIM * LPD;
    static constexpr int PADN = NODES + NODES / N;           // padded array length per element
    __host__ __device__ static constexpr int pidx(int node) { return node + node / N; }
    // (element in block, direction, line) of lane tid; el >= EPB for idle lanes
    __device__ static void lane(int tid, int &el, int &m, int &line) {
        if (FE > 0) {
            el = tid / (DIM * LINES);
            const int rem = tid - el * (DIM * LINES);
            m = rem / LINES;
            line = rem - m * LINES;
        } else {
            m = tid / LPD;
            const int r = tid - m * LPD;
            el = r / LINES;
            line = r - el * LINES;
        }
    }
};

// Launch shape of the standalone 3D Euler volume kernels: elements per block
// of the flat mapping (0: the grouped mapping; -k: grouped over k elements
// per block), the minimum number of waves
// per SIMD the register budget must allow (1: no bound), and whether the
// next partner node is loaded one pair ahead.  Measured on MI355X (n = 8
// state regrouped into n^3-node elements, against the grouped mapping):
//   n = 5:  FP64 3 elements per 4-wave block (225 of 256 lanes, grouped 50/64)
//           without the look-ahead load (126 VGPRs, 4 waves per SIMD): 1.08x;
//           FP32-split grouped without it: 1.08x;
//   n = 6:  2 elements per 4-wave block (216/256, grouped 36/64): 1.29x FP64,
//           1.22x FP32-split;
//   n = 9:  one element per 4-wave block (243/256, grouped 81/128), FP64 held
//           to 3 waves per SIMD: 2.0x;
//   n = 10: two elements per block (124 KB of LDS: one block per CU) in the
//           grouped mapping, 3 directions x 4 waves (600 of 768 lanes): a
//           flat 10-wave block of the two (600/640) ran 1.19x FP64, 1.28x
//           FP32-split and 1.18x pressure fix against the grouped 6-wave
//           block of one element, but puts 3 waves on two SIMDs and 2 on
//           the others; the 12-wave grouped block runs 3 on each, with the
//           direction a constant per wave (32 instead of 52 bytes spilled
//           at 168 VGPRs): 1.10x FP64 and pressure fix, 1.04x FP32-split
//           over the flat block;
//   n = 11: FP32-split two elements per grouped 12-wave block (726/768; 118
//           KB of LDS, 3 waves on every SIMD) against one per 6-wave block:
//           1.22x; FP64 stays at one (186 VGPRs; held to 168 so that two
//           82 KB blocks could share a CU, it spilled and ran 0.88x);
//   n = 12, 13: one element per 7- and 8-wave block (432/448, 507/512): 1.5x
//           and 1.6x (the grouped 9-wave blocks had to spill to fit).
// n = 2, 3, 4, 8 fill their waves grouped.  Flat blocks of 5 or 6 waves
// (n = 5 with 5 elements, n = 6 with 3, n = 7 with 2, n = 10 with 1) ran as
// if only one block fitted per CU, and bounding registers below the natural
// count (spilling) was slower, so n = 7 and FP64 n = 11 stay grouped over
// one element.
// With one element per block the reference values of the staging step can be
// derived by every thread instead of through LDS and a barrier: 1.03x at
// n = 8 and 1.01x at n = 12, 13 (FP64); it costs the registers that hold them
// while the stage runs, which made n = 9 spill more (no gain), the FP32-split
// form at n = 9 drop to 3 waves per SIMD (0.87x) and the pressure-fix flux at
// n = 8 exceed 168 VGPRs (0.71x), so those keep the LDS form.
struct VolumeShape {
    int fe;
    int min_waves;
    bool ahead;
    bool own_ref;
};
constexpr VolumeShape euler_volume_shape(int n, bool fp64, bool pfix = false) {
    return n == 5 ? VolumeShape{fp64 ? 3 : 0, 1, false, false}
         : n == 6 ? VolumeShape{2, 1, true, false}
         : n == 9 ? VolumeShape{1, fp64 ? 3 : 1, false, false}
         : n == 10 ? VolumeShape{-2, 1, false, false}
         : n == 11 ? VolumeShape{fp64 ? 0 : -2, 1, false, false}
         : (n == 12 || n == 13) ? VolumeShape{1, 1, false, fp64}
         : n == 8 ? VolumeShape{0, 1, true, fp64 && !pfix}
         : VolumeShape{0, 1, n <= 8, false};
}

// Padded LDS base index and stride of line `line` in direction m
// (see the padded index node + node / N).
template <int N, int DIM>
__device__ __forceinline__ void line_geometry(int m, int line, int &pbase, int &pstride,
                                              int &q0, int &q1) {
    constexpr int NN = N * N;
    if (DIM == 2) {
        q0 = line;
        q1 = 0;
        if (m == 0) { pbase = (N + 1) * q0; pstride = 1; }
        else        { pbase = q0;           pstride = N + 1; }
    } else {
        q0 = line % N;
        q1 = line / N;
        if (m == 0)      { pbase = (N + 1) * q0 + (NN + N) * q1; pstride = 1; }
        else if (m == 1) { pbase = q0 + (NN + N) * q1;           pstride = N + 1; }
        else             { pbase = q0 + (N + 1) * q1;            pstride = NN + N; }
    }
}

// Compiler fences.  pin(x) makes x opaque at this point in program order: the
// value must be computed here (it cannot be sunk into a branch) and later
// loads indexed by it cannot be merged with or hoisted above earlier ones.
template <class T>
__device__ __forceinline__ T pin(T x) {
    asm volatile("" : "+v"(x));
    return x;
}

// A wave-uniform double moved to scalar registers (both halves read from the
// first active lane), so constants used by every pair need no vector
// registers and are not rebuilt from literals at each use.
__device__ __forceinline__ double uniform_f64(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// 1/x to (about) one ulp from the hardware estimate r (relative error
// |e| < 2^-22, e = 1 - x r): 1/x = r / (1 - e) = r (1 + e + e^2 + O(e^3)),
// so one third-order correction r + r (e + e^2) replaces two Newton steps
// (three FMAs instead of four; the dropped e^3 is below 2^-66).
__device__ __forceinline__ double rcp_fine(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, __builtin_fma(e, e, e), r);
}

// ln(u + e) for a normal u > 0 and a correction |e| <= ulp(u), to about one
// ulp, without a library call.  u = 2^k m with m in [sqrt(1/2), sqrt(2));
// ln(u + e) = k ln 2 + ln m + e/u.  With f = m - 1 (exact) and s = f/(2 + f),
// ln m = 2 atanh(s) = f - f^2/2 + s (f^2/2 + R(s^2)), R(z) = sum_j 2 z^j/(2j+1)
// (|s| <= 0.1716, so nine terms leave a truncation below 1e-17 of ln m); the
// f - f^2/2 grouping keeps the rounding of s and R out of the leading terms.
// ln 2 is split so that k * kLn2Hi is exact for |k| < 2^11.  FINE_CORR
// refines the reciprocal of e/u to full precision: needed when e is
// comparable to the result (ln(1 + x) for |x| near eps), not when only the
// absolute error matters (e/u <= 2^-52, so a 2^-22 reciprocal estimate
// leaves an error below 2^-74).
constexpr double kLn2Hi = 0.6931471805598903;      // 42 leading bits of ln 2
constexpr double kLn2Lo = 5.497923018708371e-14;   // ln 2 - kLn2Hi
constexpr double kSqrtHalf = 0.7071067811865476;

template <bool FINE_CORR>
__device__ __forceinline__ double log_core(double u, double e) {
    int k = __builtin_amdgcn_frexp_exp(u);
    double m = __builtin_amdgcn_frexp_mant(u);     // u = m 2^k, m in [0.5, 1)
    if (m < kSqrtHalf) {
        m = m + m;
        k -= 1;
    }
    const double f = m - 1.0;
    const double s = f * rcp_fine(2.0 + f);
    const double z = s * s;
    double R = 2.0 / 19.0;
    R = __builtin_fma(R, z, 2.0 / 17.0);
    R = __builtin_fma(R, z, 2.0 / 15.0);
    R = __builtin_fma(R, z, 2.0 / 13.0);
    R = __builtin_fma(R, z, 2.0 / 11.0);
    R = __builtin_fma(R, z, 2.0 / 9.0);
    R = __builtin_fma(R, z, 2.0 / 7.0);
    R = __builtin_fma(R, z, 2.0 / 5.0);
    R = __builtin_fma(R, z, 2.0 / 3.0);
    R = R * z;
    const double hf = 0.5 * f * f;
    const double lnm = f - (hf - s * (hf + R));
    const double kd = (double)k;
    const double corr = __builtin_amdgcn_ldexp(e, -k) * (FINE_CORR ? rcp_fine(m) : __builtin_amdgcn_rcp(m));
    return __builtin_fma(kd, kLn2Hi, lnm + __builtin_fma(kd, kLn2Lo, corr));
}

// ln(1 + x) for finite x > -1, to about one ulp: 1 + x = u + e exactly
// (two-sum), then ln(u + e).
__device__ __forceinline__ double log1p_series(double x) {
    const double u = 1.0 + x;
    const double bv = u - 1.0;
    const double e = (1.0 - (u - bv)) + (x - bv);
    return log_core<true>(u, e);
}

// ln(x ix0) for positive normal x and ix0 (the reciprocal of a reference
// value x0): the product is split exactly, x ix0 = q + e (q rounded, e by
// one FMA), and ln(q + e) taken as above.  The absolute error is about
// eps |ln(x ix0)| plus the rounding of ix0, a relative error delta that
// adds the same ln(1 + delta) to the logarithm of every x against this ix0:
// differences ln(x_a ix0) - ln(x_b ix0) = ln x_a - ln x_b keep an absolute
// error of about eps (|ln(x_a/x0)| + |ln(x_b/x0)|), at any ratio x/x0.
__device__ __forceinline__ double log_ratio(double x, double ix0) {
    const double q = x * ix0;
    const double e = __builtin_fma(x, ix0, -q);
    return log_core<false>(q, e);
}

// ln x: ln(x + 0) as above for a positive x, about one ulp (subnormal x
// too: the hardware frexp normalises them); -inf at 0, +inf at +inf and NaN
// below 0 or at NaN (selects, no branch).
__device__ __forceinline__ double log_pos(double x) {
    const double r = log_core<false>(x, 0.0);
    const double inf = __builtin_inf();
    return (x > 0.0 && x < inf) ? r : (x == 0.0 ? -inf : (x == inf ? inf : __builtin_nan("")));
}

// e^x to about one ulp without a library call (Cody and Waite's reduction):
// x = k ln 2 + r with k = rint(x / ln 2) and r taken in two steps with the
// split ln 2 above (k kLn2Hi is exact for |k| < 2^11, so x is first clamped
// to [-1400, 1400], beyond which e^x is 0 or +inf in double; NaN passes),
// |r| <= ln 2 / 2 + ulp; e^r - 1 = r + r^2 P(r), P the Taylor series
// sum_{j >= 2} r^(j-2) / j! through j = 13 (the first term left out,
// r^14 / 14!, is below 5e-18), so that 1 + (e^r - 1) rounds once; e^x =
// 2^k e^r by an exact scaling, which rounds results beyond the double range
// to +inf or 0.
constexpr double kInvLn2 = 1.4426950408889634;
__device__ __forceinline__ double exp_fine(double x) {
    x = x < -1400.0 ? -1400.0 : (x > 1400.0 ? 1400.0 : x);
    const double kd = __builtin_rint(x * kInvLn2);
    double r = __builtin_fma(-kd, kLn2Hi, x);
    r = __builtin_fma(-kd, kLn2Lo, r);
    double P = 1.0 / 6227020800.0;                  // 1/13!
    P = __builtin_fma(P, r, 1.0 / 479001600.0);     // 1/12!
    P = __builtin_fma(P, r, 1.0 / 39916800.0);      // 1/11!
    P = __builtin_fma(P, r, 1.0 / 3628800.0);       // 1/10!
    P = __builtin_fma(P, r, 1.0 / 362880.0);        // 1/9!
    P = __builtin_fma(P, r, 1.0 / 40320.0);         // 1/8!
    P = __builtin_fma(P, r, 1.0 / 5040.0);          // 1/7!
    P = __builtin_fma(P, r, 1.0 / 720.0);           // 1/6!
    P = __builtin_fma(P, r, 1.0 / 120.0);           // 1/5!
    P = __builtin_fma(P, r, 1.0 / 24.0);            // 1/4!
    P = __builtin_fma(P, r, 1.0 / 6.0);             // 1/3!
    P = __builtin_fma(P, r, 0.5);                   // 1/2!
    const double em1 = __builtin_fma(r * r, P, r);  // e^r - 1
    return __builtin_amdgcn_ldexp(1.0 + em1, (int)kd);
}

// ---------------------------------------------------------------------------
// Scalar fluxes (1 variable, one stored quantity per node).
// ---------------------------------------------------------------------------
struct ScalarNode {
    double u;
};

template <int KIND>  // 0 = Burgers EC, 2 = product
struct ScalarFlux {
    using Real = double;
    static constexpr int NV = 1;
    static constexpr int NS = 1;
    static constexpr int NX = 0;  // extra per-node input arrays (none)
    using Node = ScalarNode;

    static constexpr int NREF = 0;
    __device__ static void make_ref(const double *, double, double *) {}
    __device__ static void stage(const double *uc, const double *, double, double *s) { s[0] = uc[0]; }

    __device__ static Node load(const double *lds, int arrstride, int idx, int) {
        (void)arrstride;
        return Node{lds[idx]};
    }
    __device__ static Node load_partner(const double *lds, int arrstride, int idx, int m) {
        return load(lds, arrstride, idx, m);
    }

    struct Consts {};
    __device__ static Consts consts(double) { return Consts{}; }

    __device__ static void pair(const Node &A, const Node &C, const Consts &, double *F) {
        if (KIND == 0)
            F[0] = (A.u * A.u + A.u * C.u + C.u * C.u) * (1.0 / 6.0);
        else
            F[0] = A.u * C.u;
    }

    __device__ static void diag(const Node &A, double, double *F) {
        if (KIND == 0)
            F[0] = 0.5 * A.u * A.u;
        else
            F[0] = A.u * A.u;
    }

    // LDS output array of accumulator k for direction m.
    __device__ static int out_array(int, int) { return 0; }
};

// ---------------------------------------------------------------------------
// Chandrashekar's entropy-conserving, kinetic-energy-preserving Euler flux,
// FP64.  Stored per node: half the density r = rho/2 (a sum of two stored
// values is the mean {{rho}}), half velocities w = v/2 (a sum is a mean
// velocity), beta = rho/(2p), and the logarithms
//     lr = ln(rho / rho_0) / 2,     lb = cg ln(beta / beta_0),
// cg = 1/(2(gamma-1)), against the element's first node (rho_0, beta_0;
// log_ratio), so that their rounding error is about eps |ln(a / a_0)|,
// i.e. scales with the element's own variation rather than with |ln a|.  A
// lane works in the frame of its line, (n, t1, t2) = (m, m+1, m+2) mod 3, so
// the flux code has no direction branches; accumulators are (rho, n-, t1-,
// t2-momentum, E).
//
// Logarithmic means a^ln = (a - b)/(ln a - ln b) are carried as a fraction
// N/D.  For rho, in halves (s = r_a + r_b, d = r_a - r_b, u = d^2/s^2):
//   direct:        N = d,        D = lr_a - lr_b  (= (ln rho_a - ln rho_b)/2)
//   near-equal:    N = s^3,      D = s^2 + d^2 (1/3 + u/5),
// for beta (s = b_a + b_b, d = b_a - b_b), carrying cg / beta^ln = D/N:
//   direct:        N = d,        D = lb_a - lb_b
//   near-equal:    N = s^3/2,    D = cg (s^2 + d^2 (1/3 + u/5)).
// The near-equal form is s times the series of f/atanh(f), f = d/s (the
// truncation u^3/7 is below 1.5e-19 for u < 1e-6; exact equality gives the
// mean exactly); it is taken when |ln a - ln b| < 2e-3, i.e.
// |f| = tanh(|ln a - ln b| / 2) < ~1e-3, tested on the stored logarithms
// (one compare, no multiply).  The direct form's relative error is about
// eps (|ln(a/a_0)| + |ln(b/a_0)| + 2) / |ln a - ln b|: below about 1e-13 at
// the switch for an element whose values stay within a factor e of its first
// node's, and growing with the logarithm of the in-element ratio (about
// 3e-12 at the switch for ratios of 1e6).  The near-equal case is a real
// branch that waves with no near-equal lane skip.
// The three quotients the flux needs -- rho^ln = Nr/Dr, cg/beta^ln = Db/Nb
// and p_hat = {{rho}}/(2{{beta}}) = s_r/s_b -- share one reciprocal
// R = 1/(Dr Nb s_b): each quotient is its numerator times R times the other
// two factors, formed as pairwise products.
// Valid for rho, beta in about [1e-30, 1e30].
//
// PFIX: Chandrashekar's flux with Ranocha's pressure fix -- the momentum
// flux takes the arithmetic pressure mean {{p}} instead of p_hat, and the
// energy flux the entropy-conservative completion,
//     F^E = F^rho [1/(2(gamma-1) beta^ln) + v_L.v_R/2] + (p_L v_nR + p_R v_nL)/2.
// Half the pressure is stored as an eighth quantity (a sum of two is {{p}});
// only rho^ln and cg/beta^ln are quotients, R = 1/(Dr Nb).
// ---------------------------------------------------------------------------
struct EulerNode {
    double r, wn, wt1, wt2, b, lr, lb, ph;
};

template <bool PFIX>
struct EulerFP64T {
    using Real = double;
    static constexpr int NV = 5;
    static constexpr bool PRESSURE_FIX = PFIX;
    static constexpr int NS = PFIX ? 8 : 7;
    static constexpr int NX = 0;
    static constexpr int NREF = 2;  // 1/rho_0, 1/beta_0
    enum { S_R = 0, S_W = 1, S_B = 4, S_LR = 5, S_LB = 6, S_P = 7 };
    using Node = EulerNode;
    // Series branch when |ln a - ln b| < kLogTau, i.e. |a - b|/(a + b) =
    // tanh(|ln a - ln b| / 2) < ~1e-3 (u = f^2 < 1e-6).
    static constexpr double kLogTau = 2e-3;

    // v, p and beta = rho/(2p) of a conserved state; returns 1/rho
    __device__ static double primitives(const double *uc, double gamma, double (&v)[3], double &p,
                                        double &beta) {
        const double r = uc[0];
        const double ir = rcp_fine(r);
        v[0] = uc[1] * ir;
        v[1] = uc[2] * ir;
        v[2] = uc[3] * ir;
        p = (gamma - 1.0) * (uc[4] - 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
        beta = 0.5 * r * rcp_fine(p);
        return ir;
    }

    // The element's reference values, from its first node's conserved state.
    __device__ static void make_ref(const double *uc, double gamma, double *ref) {
        double v[3], p, b;
        ref[0] = primitives(uc, gamma, v, p, b);
        ref[1] = rcp_fine(b);
    }

    // a1: conserved -> stored quantities (FP64, per node).
    __device__ static void stage(const double *uc, const double *ref, double gamma, double *s) {
        double v[3], p, b;
        primitives(uc, gamma, v, p, b);
        const double r = uc[0];
        s[S_R] = 0.5 * r;
        s[S_W + 0] = 0.5 * v[0];
        s[S_W + 1] = 0.5 * v[1];
        s[S_W + 2] = 0.5 * v[2];
        s[S_B] = b;
        s[S_LR] = 0.5 * log_ratio(r, ref[0]);
        s[S_LB] = (0.5 / (gamma - 1.0)) * log_ratio(b, ref[1]);
        if (PFIX) s[S_P] = 0.5 * p;
    }

    // Load node at padded index idx of one element's arrays (arrays are
    // arrstride doubles apart), rotated into the frame of direction m.
    __device__ static Node load(const double *lds, int arrstride, int idx, int m) {
        int t1 = m == 2 ? 0 : m + 1;
        int t2 = m == 0 ? 2 : m - 1;
        Node A;
        A.r = lds[S_R * arrstride + idx];
        A.wn = lds[(S_W + m) * arrstride + idx];
        A.wt1 = lds[(S_W + t1) * arrstride + idx];
        A.wt2 = lds[(S_W + t2) * arrstride + idx];
        A.b = lds[S_B * arrstride + idx];
        A.lr = lds[S_LR * arrstride + idx];
        A.lb = lds[S_LB * arrstride + idx];
        A.ph = PFIX ? lds[S_P * arrstride + idx] : 0.0;
        return A;
    }

    __device__ static Node load_partner(const double *lds, int arrstride, int idx, int m) {
        return load(lds, arrstride, idx, m);
    }

    // Constants of the pair flux, in scalar registers for the whole kernel
    // (64-bit values that are not inline operands would otherwise be rebuilt
    // for every pair).  thr_r is on the halved ln rho, thr_b carries the cg
    // folded into the stored ln beta.
    struct Consts {
        double cg, c3, c5, thr_r, thr_b;
    };
    __device__ static Consts consts(double cg) {
        return Consts{uniform_f64(cg), uniform_f64(1.0 / 3.0), uniform_f64(0.2), uniform_f64(0.5 * kLogTau),
                      uniform_f64(kLogTau * cg)};
    }

    // The three quotients of a pair: rho^ln, cg/beta^ln and p_hat.
    __device__ static void means(const Node &A, const Node &C, const Consts &K, double &rho_ln, double &cgib,
                                 double &phat) {
        const double sr = A.r + C.r, dr = A.r - C.r;   // {{rho}}, (rho_a - rho_b)/2
        const double sb = A.b + C.b, db = A.b - C.b;   // 2 {{beta}}, beta_a - beta_b
        double Nr = dr, Dr = A.lr - C.lr;
        double Nb = db, Db = A.lb - C.lb;
        if (__builtin_fabs(Dr) < K.thr_r) {  // near-equal densities: series
            const double dr2 = dr * dr, sr2 = sr * sr;
            const double u = dr2 * __builtin_amdgcn_rcp(sr2);
            Nr = pin(sr * sr2);
            Dr = __builtin_fma(dr2, __builtin_fma(u, K.c5, K.c3), sr2);
        }
        if (__builtin_fabs(Db) < K.thr_b) {  // near-equal beta: series, times cg
            const double db2 = db * db, sb2 = sb * sb;
            const double u = db2 * __builtin_amdgcn_rcp(sb2);
            Nb = pin(0.5 * sb * sb2);
            Db = K.cg * __builtin_fma(db2, __builtin_fma(u, K.c5, K.c3), sb2);
        }
        if (PFIX) {  // no p_hat: R = 1/(Dr Nb)
            const double R = rcp_fine(Dr * Nb);
            rho_ln = Nr * (Nb * R);
            cgib = Db * (Dr * R);
            phat = 0.0;
        } else {
            const double P1 = Nb * sb, P2 = Dr * sb, P3 = Dr * Nb;
            const double R = rcp_fine(Dr * P1);
            rho_ln = Nr * (P1 * R);
            cgib = Db * (P2 * R);       // cg / beta^ln
            phat = sr * (P3 * R);       // {{rho}} / (2 {{beta}})
        }
    }

    // a4: two-point flux f_n(A, C) in the line frame (cg is folded into lb).
    __device__ static void pair(const Node &A, const Node &C, const Consts &K, double *F) {
        double rho_ln, cgib, phat;
        means(A, C, K, rho_ln, cgib, phat);
        const double vn = A.wn + C.wn, v1 = A.wt1 + C.wt1, v2 = A.wt2 + C.wt2;     // {{v}}
        const double ww = __builtin_fma(A.wn, C.wn, __builtin_fma(A.wt1, C.wt1, A.wt2 * C.wt2));  // v_L.v_R / 4
        const double F0 = rho_ln * vn;
        F[0] = F0;
        F[2] = F0 * v1;
        F[3] = F0 * v2;
        if (PFIX) {
            // {{p}} = ph_a + ph_c; (p_a v_nc + p_c v_na)/2 = 2 (ph_a w_nc + ph_c w_na)
            const double work = __builtin_fma(A.ph, C.wn, C.ph * A.wn);
            F[1] = __builtin_fma(F0, vn, A.ph + C.ph);
            F[4] = __builtin_fma(F0, __builtin_fma(2.0, ww, cgib), work + work);
        } else {
            F[1] = __builtin_fma(F0, vn, phat);
            // F^E = F^rho [1/(2(gamma-1) beta^ln) + v_L.v_R/2] + p_hat {{v_n}}
            F[4] = __builtin_fma(F0, __builtin_fma(2.0, ww, cgib), phat * vn);
        }
    }

    // Physical flux f_n(u) (the pair flux at equal states), from stored data
    // (r = rho/2, w = v/2): p = r/beta, rho v_n = 4 r w_n,
    // (E + p) v_n = 2 w_n (gamma/(gamma-1) p + 4 r |w|^2).
    __device__ static void diag(const Node &A, double gamma, double *F) {
        const double p = PFIX ? A.ph + A.ph : A.r * rcp_fine(A.b);
        const double rw = A.r * A.wn;
        const double F0 = 4.0 * rw;
        const double G = 8.0 * rw;                       // rho v_n * 2
        const double q = __builtin_fma(A.wn, A.wn, __builtin_fma(A.wt1, A.wt1, A.wt2 * A.wt2));
        F[0] = F0;
        F[1] = __builtin_fma(G, A.wn, p);
        F[2] = G * A.wt1;
        F[3] = G * A.wt2;
        F[4] = (A.wn + A.wn) * __builtin_fma(4.0 * A.r, q, (gamma / (gamma - 1.0)) * p);
    }

    // Conserved-variable array of accumulator k in direction m's frame.
    __device__ static int out_array(int k, int m) {
        if (k == 0 || k == 4) return k;
        int comp = m + (k - 1);
        if (comp >= 3) comp -= 3;
        return 1 + comp;
    }
};
using EulerFP64 = EulerFP64T<false>;
using EulerPFixFP64 = EulerFP64T<true>;

// ---------------------------------------------------------------------------
// FP32-split form of the Euler flux: stored quantities, pair and diagonal
// fluxes and the line sums are FP32; the direction sum is FP64 (in the
// kernel).  The per-node logarithms, relative to the element's first node as
// in the FP64 form, are taken in FP64 of the stored (FP32) rho and beta and
// kept as two FP32 words (hi + lo), so ln a - ln b of two close states keeps
// ~1e-16 absolute accuracy and the direct form
// (a - b)/(ln a - ln b) stays accurate to FP32 rounding until a and b are
// within about 1e-6 relative.  Below that (|ln a - ln b| < 2e-6, tested on
// the hi + lo differences, exact equality included) the logarithmic mean is
// evaluated in FP64 by the series and rounded.
// ---------------------------------------------------------------------------
struct EulerNodeF {
    float r, wn, wt1, wt2, b, p, lrh, lrl, lbh, lbl;
};

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// (a - b)/(ln a - ln b) for a, b within 1e-6 relative, in FP64:
// (a + b)/2 (1 - u/3), u = ((a-b)/(a+b))^2 (the next term, 4u^2/45, is below 1e-24).
__device__ __forceinline__ double logmean_near64(float a, float b) {
    const double A = a, B = b;
    const double s = A + B, d = A - B;  // exact for FP32 inputs
    const double u = (d * d) * rcp_fine(s * s);
    return 0.5 * s * __builtin_fma(u, -1.0 / 3.0, 1.0);
}

// 1 / logmean(a, b) for a, b within 1e-6 relative, in FP64: 2 (1 + u/3) / (a + b).
__device__ __forceinline__ double inv_logmean_near64(float a, float b) {
    const double A = a, B = b;
    const double s = A + B, d = A - B;
    const double rs = rcp_fine(s);
    const double f = d * rs;
    return 2.0 * rs * __builtin_fma(f * f, 1.0 / 3.0, 1.0);
}

struct EulerFP32Split {
    using Real = float;
    static constexpr int NV = 5;
    static constexpr int NS = 10;
    static constexpr int NX = 0;
    enum { S_R = 0, S_W = 1, S_B = 4, S_P = 5, S_LRH = 6, S_LRL = 7, S_LBH = 8, S_LBL = 9 };
    using Node = EulerNodeF;
    // FP64 series below |ln a - ln b| = 2e-6, i.e. |a - b| < ~1e-6 (a + b)
    static constexpr float kLogTau = 2e-6f;

    // a1 in FP64, stored rounded to FP32 in the FP64 form's halved layout
    // (r = rho/2, w = v/2, lr = ln(rho/rho_0)/2 as hi + lo); the logarithms
    // are of the stored values, against the element's first node (log_ratio).
    static constexpr int NREF = 2;  // 1/rho_0, 1/beta_0 (of the FP32-rounded values)
    __device__ static void make_ref(const double *uc, double gamma, double *ref) {
        double v[3], p, b;
        EulerFP64::primitives(uc, gamma, v, p, b);
        ref[0] = rcp_fine((double)(float)(0.5 * uc[0]));
        ref[1] = rcp_fine((double)(float)b);
    }

    __device__ static void stage(const double *uc, const double *ref, double gamma, float *s) {
        double v[3], p, b;
        EulerFP64::primitives(uc, gamma, v, p, b);
        const float rf = (float)(0.5 * uc[0]), bf = (float)b;
        s[S_R] = rf;
        s[S_W + 0] = (float)(0.5 * v[0]);
        s[S_W + 1] = (float)(0.5 * v[1]);
        s[S_W + 2] = (float)(0.5 * v[2]);
        s[S_B] = bf;
        s[S_P] = (float)p;
        const double lr = 0.5 * log_ratio((double)rf, ref[0]);
        const double lb = (0.5 / (gamma - 1.0)) * log_ratio((double)bf, ref[1]);
        const float lrh = (float)lr, lbh = (float)lb;
        s[S_LRH] = lrh;
        s[S_LRL] = (float)(lr - (double)lrh);
        s[S_LBH] = lbh;
        s[S_LBL] = (float)(lb - (double)lbh);
    }

    __device__ static Node load(const float *lds, int arrstride, int idx, int m) {
        const int t1 = m == 2 ? 0 : m + 1;
        const int t2 = m == 0 ? 2 : m - 1;
        Node A;
        A.r = lds[S_R * arrstride + idx];
        A.wn = lds[(S_W + m) * arrstride + idx];
        A.wt1 = lds[(S_W + t1) * arrstride + idx];
        A.wt2 = lds[(S_W + t2) * arrstride + idx];
        A.b = lds[S_B * arrstride + idx];
        A.p = lds[S_P * arrstride + idx];
        A.lrh = lds[S_LRH * arrstride + idx];
        A.lrl = lds[S_LRL * arrstride + idx];
        A.lbh = lds[S_LBH * arrstride + idx];
        A.lbl = lds[S_LBL * arrstride + idx];
        return A;
    }

    __device__ static Node load_partner(const float *lds, int arrstride, int idx, int m) {
        Node A = load(lds, arrstride, idx, m);
        return A;
    }

    struct Consts {
        float cg, thr_r, thr_b;
    };
    __device__ static Consts consts(double cg) {
        return Consts{(float)cg, 0.5f * kLogTau, (float)(kLogTau * cg)};
    }

    // As the FP64 form, in FP32 (halved density and logarithm, one
    // reciprocal for the three quotients); the switch to the FP64 series is
    // tested on the (hi + lo) logarithm differences.
    __device__ static void pair(const Node &A, const Node &C, const Consts &K, float *F) {
        const float dr = A.r - C.r, sr = A.r + C.r;   // (rho_a - rho_c)/2, {{rho}}
        const float db = A.b - C.b, sb = A.b + C.b;
        float Nr = dr, Dr = pin((A.lrh - C.lrh) + (A.lrl - C.lrl));
        float Nb = db, Db = pin((A.lbh - C.lbh) + (A.lbl - C.lbl));
        if (__builtin_fabsf(Dr) < K.thr_r) {  // near-identical densities: FP64 series of the halves,
            Nr = (float)logmean_near64(A.r, C.r);  // rho^ln / 2, over a halved log difference of 1/2
            Dr = 0.5f;
        }
        if (__builtin_fabsf(Db) < K.thr_b) {  // near-identical beta: FP64 series
            Db = (float)((double)K.cg * inv_logmean_near64(A.b, C.b));
            Nb = 1.0f;
        }
        const float P1 = Nb * sb, P2 = Dr * sb, P3 = Dr * Nb;
        const float R = rcpf(Dr * P1);
        const float rho_ln = Nr * (P1 * R);
        const float cgib = Db * (P2 * R);
        const float phat = sr * (P3 * R);

        const float vn = A.wn + C.wn, v1 = A.wt1 + C.wt1, v2 = A.wt2 + C.wt2;
        const float ww = __builtin_fmaf(A.wn, C.wn, __builtin_fmaf(A.wt1, C.wt1, A.wt2 * C.wt2));
        const float F0 = rho_ln * vn;
        F[0] = F0;
        F[1] = __builtin_fmaf(F0, vn, phat);
        F[2] = F0 * v1;
        F[3] = F0 * v2;
        F[4] = __builtin_fmaf(F0, __builtin_fmaf(2.0f, ww, cgib), phat * vn);
    }

    // physical flux from the stored halves: rho v_n = 4 r w_n,
    // (E + p) v_n = 2 w_n (gamma/(gamma-1) p + 4 r |w|^2)
    __device__ static void diag(const Node &A, double gamma, float *F) {
        const float rw = A.r * A.wn;
        const float G = 8.0f * rw;
        const float q = __builtin_fmaf(A.wn, A.wn, __builtin_fmaf(A.wt1, A.wt1, A.wt2 * A.wt2));
        F[0] = 4.0f * rw;
        F[1] = __builtin_fmaf(G, A.wn, A.p);
        F[2] = G * A.wt1;
        F[3] = G * A.wt2;
        F[4] = (A.wn + A.wn) * __builtin_fmaf(4.0f * A.r, q, (float)(gamma / (gamma - 1.0)) * A.p);
    }

    __device__ static int out_array(int k, int m) { return EulerFP64::out_array(k, m); }
};


// ---------------------------------------------------------------------------
// Curvilinear Euler (FP64): the metric-averaged two-point flux in reference
// direction m,
//     F_m(u_i, u_j) = sum_k f_k(u_i, u_j) n_k,   n = (Ja^m(i) + Ja^m(j)) / 2,
// with Ja^m_k = J d xi^m / d x_k the contravariant metric terms (the 9 extra
// per-node inputs, stored halved).  Since the Chandrashekar flux is linear in
// the direction, the sum is one flux with normal velocity {{v}} . n and
// pressure term p_hat n:
//     F^rho = rho^ln {{v}}.n,  F^(rho v_k) = F^rho {{v_k}} + p_hat n_k,
//     F^E = F^rho [1/(2(gamma-1) beta^ln) + v_L.v_R/2] + p_hat {{v}}.n .
// With PFIX (the pressure fix) the pressure terms become {{p}} n_k and
// (p_L v_R.n + p_R v_L.n)/2.
// Velocities and results stay Cartesian (no rotation into a line frame).
// ---------------------------------------------------------------------------
struct EulerCurvNode {
    double r, w0, w1, w2, b, lr, lb, ph, n0, n1, n2;
};

template <bool PFIX>
struct EulerCurvT {
    using Base = EulerFP64T<PFIX>;
    using Real = double;
    static constexpr int NV = 5;
    static constexpr int NX = 9;             // Ja^m_k, m-major
    static constexpr int NS = Base::NS + 9;  // the Cartesian flux's stored values (unrotated) + 9 halved metric terms
    static constexpr int NREF = Base::NREF;
    enum { S_R = 0, S_W = 1, S_B = 4, S_LR = 5, S_LB = 6, S_P = 7, S_N = Base::NS };
    using Node = EulerCurvNode;
    using Consts = typename Base::Consts;

    __device__ static void make_ref(const double *uc, double gamma, double *ref) { Base::make_ref(uc, gamma, ref); }
    // uc: the 5 conserved variables, then the 9 metric terms
    __device__ static void stage(const double *uc, const double *ref, double gamma, double *s) {
        Base::stage(uc, ref, gamma, s);
#pragma unroll
        for (int j = 0; j < NX; ++j) s[S_N + j] = 0.5 * uc[NV + j];
    }
    __device__ static Node load(const double *lds, int arrstride, int idx, int m) {
        Node A;
        A.r = lds[S_R * arrstride + idx];
        A.w0 = lds[(S_W + 0) * arrstride + idx];
        A.w1 = lds[(S_W + 1) * arrstride + idx];
        A.w2 = lds[(S_W + 2) * arrstride + idx];
        A.b = lds[S_B * arrstride + idx];
        A.lr = lds[S_LR * arrstride + idx];
        A.lb = lds[S_LB * arrstride + idx];
        A.ph = PFIX ? lds[S_P * arrstride + idx] : 0.0;
        A.n0 = lds[(S_N + 3 * m + 0) * arrstride + idx];
        A.n1 = lds[(S_N + 3 * m + 1) * arrstride + idx];
        A.n2 = lds[(S_N + 3 * m + 2) * arrstride + idx];
        return A;
    }
    __device__ static Node load_partner(const double *lds, int arrstride, int idx, int m) {
        return load(lds, arrstride, idx, m);
    }
    __device__ static Consts consts(double cg) { return Base::consts(cg); }

    __device__ static void pair(const Node &A, const Node &C, const Consts &K, double *F) {
        double rho_ln, cgib, phat;
        Base::means(EulerNode{A.r, 0, 0, 0, A.b, A.lr, A.lb, 0}, EulerNode{C.r, 0, 0, 0, C.b, C.lr, C.lb, 0}, K,
                    rho_ln, cgib, phat);
        const double v0 = A.w0 + C.w0, v1 = A.w1 + C.w1, v2 = A.w2 + C.w2;     // {{v}}
        const double n0 = A.n0 + C.n0, n1 = A.n1 + C.n1, n2 = A.n2 + C.n2;     // averaged Ja^m
        const double vn = __builtin_fma(v0, n0, __builtin_fma(v1, n1, v2 * n2));
        const double ww = __builtin_fma(A.w0, C.w0, __builtin_fma(A.w1, C.w1, A.w2 * C.w2));
        const double F0 = rho_ln * vn;
        const double X = __builtin_fma(2.0, ww, cgib);
        F[0] = F0;
        if (PFIX) {
            // {{p}} = ph_a + ph_c; (p_a v_c.n + p_c v_a.n)/2 = 2 (ph_a w_c.n + ph_c w_a.n)
            const double pavg = A.ph + C.ph;
            const double wan = __builtin_fma(A.w0, n0, __builtin_fma(A.w1, n1, A.w2 * n2));
            const double wcn = __builtin_fma(C.w0, n0, __builtin_fma(C.w1, n1, C.w2 * n2));
            const double work = __builtin_fma(A.ph, wcn, C.ph * wan);
            F[1] = __builtin_fma(F0, v0, pavg * n0);
            F[2] = __builtin_fma(F0, v1, pavg * n1);
            F[3] = __builtin_fma(F0, v2, pavg * n2);
            F[4] = __builtin_fma(F0, X, work + work);
        } else {
            F[1] = __builtin_fma(F0, v0, phat * n0);
            F[2] = __builtin_fma(F0, v1, phat * n1);
            F[3] = __builtin_fma(F0, v2, phat * n2);
            F[4] = __builtin_fma(F0, X, phat * vn);
        }
    }

    // physical flux f(u) . Ja^m at the node (r = rho/2, w = v/2, halved metric)
    __device__ static void diag(const Node &A, double gamma, double *F) {
        const double p = PFIX ? A.ph + A.ph : A.r * rcp_fine(A.b);
        const double v0 = A.w0 + A.w0, v1 = A.w1 + A.w1, v2 = A.w2 + A.w2;
        const double n0 = A.n0 + A.n0, n1 = A.n1 + A.n1, n2 = A.n2 + A.n2;
        const double vn = __builtin_fma(v0, n0, __builtin_fma(v1, n1, v2 * n2));
        const double rvn = (A.r + A.r) * vn;
        const double q = __builtin_fma(v0, v0, __builtin_fma(v1, v1, v2 * v2));
        F[0] = rvn;
        F[1] = __builtin_fma(rvn, v0, p * n0);
        F[2] = __builtin_fma(rvn, v1, p * n1);
        F[3] = __builtin_fma(rvn, v2, p * n2);
        F[4] = vn * __builtin_fma(gamma / (gamma - 1.0), p, A.r * q);
    }

    __device__ static int out_array(int k, int) { return k; }
};
using EulerCurvFP64 = EulerCurvT<false>;
using EulerCurvPFixFP64 = EulerCurvT<true>;

}  // namespace dev
}  // namespace sfhad
