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
};

template <int N, int DIM>
struct Geom {
    static constexpr int LINES = DIM == 3 ? N * N : N;       // lines per direction per element
    static constexpr int NODES = LINES * N;                  // n^d
    static constexpr int EPB = LINES >= 64 ? 1 : 64 / LINES; // elements per block
    static constexpr int LPD = ((EPB * LINES + 63) / 64) * 64;  // lanes per direction group
    static constexpr int THREADS = DIM * LPD;
    static constexpr int PADN = NODES + NODES / N;           // padded array length per element
    __host__ __device__ static constexpr int pidx(int node) { return node + node / N; }
};

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

// 1/x to (about) one ulp: hardware reciprocal estimate plus two Newton steps.
__device__ __forceinline__ double rcp_fine(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// 1/x to ~1e-14 relative: estimate plus one Newton step (only used where the
// quotient feeds a correction term of size <= 1e-4 relative).
__device__ __forceinline__ double rcp_coarse(double x) {
    double r = __builtin_amdgcn_rcp(x);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
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
    using Node = ScalarNode;

    __device__ static void stage(const double *uc, double, double *s) { s[0] = uc[0]; }

    __device__ static Node load(const double *lds, int arrstride, int idx, int) {
        (void)arrstride;
        return Node{lds[idx]};
    }

    __device__ static void pair(const Node &A, const Node &C, double, double *F) {
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
// FP64.  Stored per node: rho, half velocities w = v/2 (so that a sum of two
// stored values is a mean velocity), beta = rho / (2 p), ln rho, ln beta.  A
// lane works in the frame of its line: (n, t1, t2) = (m, m+1, m+2) mod 3, so
// the flux code has no direction branches; accumulators are (rho,
// n-momentum, t1-momentum, t2-momentum, energy).
//
// Logarithmic means a^ln = (a - b)/(ln a - ln b) are carried as a fraction
// N/D.  With s = a + b, d = a - b and u = d^2/s^2:
//   u >= 1e-4:  N = d,          D = ln a - ln b          (per-node logs)
//   u <  1e-4:  N = s^3/2,      D = s^2 + d^2 (1/3 + u/5 + u^2/7)
// the second being s^2 times the series 1 + u/3 + u^2/5 + u^3/7 of
// atanh(f)/f, f = d/s (truncation < 1.2e-17 relative; u only enters the
// terms of size u^2, so a single hardware reciprocal estimate suffices for
// it).  The form is chosen per pair by selects, not branches.  The three
// quotients the flux needs -- rho^ln = Nr/Dr, 1/beta^ln = Db/Nb and
// p_hat = {{rho}}/(2{{beta}}) = (s_rho/2)/s_beta -- share one reciprocal
// 1/(Dr Nb s_beta).  Valid for rho, beta in about [1e-30, 1e30] (the
// products of up to six such factors stay in range).
// ---------------------------------------------------------------------------
struct EulerNode {
    double r, wn, wt1, wt2, b, lr, lb;
};

struct EulerFP64 {
    using Real = double;
    static constexpr int NV = 5;
    static constexpr int NS = 7;
    enum { S_R = 0, S_W = 1, S_B = 4, S_LR = 5, S_LB = 6 };
    using Node = EulerNode;
    static constexpr double kTau = 1e-4;

    // a1: conserved -> stored quantities (FP64, per node).
    __device__ static void stage(const double *uc, double gamma, double *s) {
        double r = uc[0];
        double ir = rcp_fine(r);
        double v0 = uc[1] * ir, v1 = uc[2] * ir, v2 = uc[3] * ir;
        double p = (gamma - 1.0) * (uc[4] - 0.5 * r * (v0 * v0 + v1 * v1 + v2 * v2));
        double b = 0.5 * r * rcp_fine(p);
        s[S_R] = r;
        s[S_W + 0] = 0.5 * v0;
        s[S_W + 1] = 0.5 * v1;
        s[S_W + 2] = 0.5 * v2;
        s[S_B] = b;
        s[S_LR] = log(r);
        s[S_LB] = log(b);
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
        return A;
    }

    // a4: two-point flux f_n(A, C) in the line frame.  cg = 1 / (2 (gamma - 1)).
    __device__ static void pair(const Node &A, const Node &C, double cg, double *F) {
        const double dr = A.r - C.r, sr = A.r + C.r;
        const double db = A.b - C.b, sb = A.b + C.b;
        const double dr2 = dr * dr, sr2 = sr * sr, db2 = db * db, sb2 = sb * sb;
        const double ur = dr2 * __builtin_amdgcn_rcp(sr2);
        const double ub = db2 * __builtin_amdgcn_rcp(sb2);
        const bool near_r = ur < kTau, near_b = ub < kTau;
        const double hsr = 0.5 * sr, hsb = 0.5 * sb;
        // series forms (computed on every lane; selected below)
        const double Nrs = pin(hsr * sr2);
        const double Drs = pin(__builtin_fma(dr2, __builtin_fma(ur, __builtin_fma(ur, 1.0 / 7.0, 0.2), 1.0 / 3.0), sr2));
        const double Nbs = pin(hsb * sb2);
        const double Dbs = pin(__builtin_fma(db2, __builtin_fma(ub, __builtin_fma(ub, 1.0 / 7.0, 0.2), 1.0 / 3.0), sb2));
        const double dlr = pin(A.lr - C.lr), dlb = pin(A.lb - C.lb);
        const double Nr = near_r ? Nrs : dr;
        const double Dr = near_r ? Drs : dlr;
        const double Nb = near_b ? Nbs : db;
        const double Db = near_b ? Dbs : dlb;
        const double DrNb = Dr * Nb;
        const double R = rcp_fine(DrNb * sb);
        const double rho_ln = Nr * (Nb * sb) * R;
        const double ibeta_ln = Db * (Dr * sb) * R;
        const double phat = hsr * DrNb * R;

        const double vn = A.wn + C.wn, v1 = A.wt1 + C.wt1, v2 = A.wt2 + C.wt2;     // {{v}}
        const double ww = __builtin_fma(A.wn, C.wn, __builtin_fma(A.wt1, C.wt1, A.wt2 * C.wt2));  // v_L.v_R / 4
        const double F0 = rho_ln * vn;
        F[0] = F0;
        F[1] = __builtin_fma(F0, vn, phat);
        F[2] = F0 * v1;
        F[3] = F0 * v2;
        // F^E = F^rho [1/(2(gamma-1) beta^ln) + v_L.v_R/2] + p_hat {{v_n}}
        F[4] = __builtin_fma(F0, __builtin_fma(2.0, ww, cg * ibeta_ln), phat * vn);
    }

    // Physical flux f_n(u) (the pair flux at equal states), from stored data.
    __device__ static void diag(const Node &A, double gamma, double *F) {
        const double p = 0.5 * A.r * rcp_fine(A.b);
        const double vn = A.wn + A.wn, v1 = A.wt1 + A.wt1, v2 = A.wt2 + A.wt2;
        const double rvn = A.r * vn;
        const double q = __builtin_fma(vn, vn, __builtin_fma(v1, v1, v2 * v2));
        F[0] = rvn;
        F[1] = __builtin_fma(rvn, vn, p);
        F[2] = rvn * v1;
        F[3] = rvn * v2;
        // (E + p) v_n with E + p = gamma/(gamma-1) p + rho |v|^2 / 2
        F[4] = vn * __builtin_fma(gamma / (gamma - 1.0), p, 0.5 * A.r * q);
    }

    // Conserved-variable array of accumulator k in direction m's frame.
    __device__ static int out_array(int k, int m) {
        if (k == 0 || k == 4) return k;
        int comp = m + (k - 1);
        if (comp >= 3) comp -= 3;
        return 1 + comp;
    }
};

// ---------------------------------------------------------------------------
// FP32-split form of the Euler flux: the stored quantities, the pair and
// diagonal fluxes and the line sums are FP32; a logarithmic mean whose
// arguments are near-equal (u = ((a-b)/(a+b))^2 < 1e-4, tested in FP32) is
// evaluated from the FP32 arguments in FP64 with the series, then rounded;
// the direction sum is FP64 (in the kernel).  The per-node logarithms are
// taken in FP64 and rounded, so ln a - ln b carries only the rounding of the
// two stored values.
// ---------------------------------------------------------------------------
struct EulerNodeF {
    float r, vn, vt1, vt2, b, lr, lb;
};

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// (a - b) / (ln a - ln b) for near-equal a, b: FP64 series
// (a + b)/2 * (1 - u/3 - 4u^2/45 - 44u^3/945), u = ((a-b)/(a+b))^2 < 1e-4
// (the reciprocal of 1 + u/3 + u^2/5 + u^3/7; truncation < 1e-17).
__device__ __forceinline__ float logmean_near64(float a, float b) {
    double A = a, B = b;
    double s = A + B, d = A - B;  // exact for FP32 inputs
    double f = d * rcp_coarse(s);
    double u = f * f;
    double P = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, -44.0 / 945.0, -4.0 / 45.0), -1.0 / 3.0), 1.0);
    return (float)(0.5 * s * P);
}

// 1 / logmean(a, b) for near-equal a, b: FP64 2 (1 + u/3 + u^2/5 + u^3/7) / (a + b).
__device__ __forceinline__ float inv_logmean_near64(float a, float b) {
    double A = a, B = b;
    double s = A + B, d = A - B;
    double rs = rcp_fine(s);
    double f = d * rs;
    double u = f * f;
    double S = __builtin_fma(u, __builtin_fma(u, __builtin_fma(u, 1.0 / 7.0, 1.0 / 5.0), 1.0 / 3.0), 1.0);
    return (float)(2.0 * rs * S);
}

struct EulerFP32Split {
    using Real = float;
    static constexpr int NV = 5;
    static constexpr int NS = 7;
    enum { S_R = 0, S_V = 1, S_B = 4, S_LR = 5, S_LB = 6 };
    using Node = EulerNodeF;
    static constexpr float kTau = 1e-4f;

    // a1 in FP64, stored rounded to FP32.
    __device__ static void stage(const double *uc, double gamma, float *s) {
        double r = uc[0];
        double ir = 1.0 / r;
        double v0 = uc[1] * ir, v1 = uc[2] * ir, v2 = uc[3] * ir;
        double p = (gamma - 1.0) * (uc[4] - 0.5 * r * (v0 * v0 + v1 * v1 + v2 * v2));
        double b = 0.5 * r / p;
        float rf = (float)r, bf = (float)b;
        s[S_R] = rf;
        s[S_V + 0] = (float)v0;
        s[S_V + 1] = (float)v1;
        s[S_V + 2] = (float)v2;
        s[S_B] = bf;
        s[S_LR] = (float)log((double)rf);  // logs of the stored (rounded) values
        s[S_LB] = (float)log((double)bf);
    }

    __device__ static Node load(const float *lds, int arrstride, int idx, int m) {
        int t1 = m == 2 ? 0 : m + 1;
        int t2 = m == 0 ? 2 : m - 1;
        Node A;
        A.r = lds[S_R * arrstride + idx];
        A.vn = lds[(S_V + m) * arrstride + idx];
        A.vt1 = lds[(S_V + t1) * arrstride + idx];
        A.vt2 = lds[(S_V + t2) * arrstride + idx];
        A.b = lds[S_B * arrstride + idx];
        A.lr = lds[S_LR * arrstride + idx];
        A.lb = lds[S_LB * arrstride + idx];
        return A;
    }

    __device__ static void pair(const Node &A, const Node &C, float cg, float *F) {
        float dr = A.r - C.r, sr = A.r + C.r;
        float db = A.b - C.b, sb = A.b + C.b;
        bool near_r = dr * dr < kTau * (sr * sr);
        bool near_b = db * db < kTau * (sb * sb);
        float rho_ln = dr * rcpf(A.lr - C.lr);
        float ibeta_ln = (A.lb - C.lb) * rcpf(db);
        if (near_r) rho_ln = logmean_near64(A.r, C.r);
        if (near_b) ibeta_ln = inv_logmean_near64(A.b, C.b);
        float phat = 0.5f * sr * rcpf(sb);

        float Vn = A.vn + C.vn, V1 = A.vt1 + C.vt1, V2 = A.vt2 + C.vt2;
        float vv = A.vn * C.vn + A.vt1 * C.vt1 + A.vt2 * C.vt2;
        float Fr = 0.5f * rho_ln * Vn;
        float hFr = 0.5f * Fr;
        F[0] = Fr;
        F[1] = __builtin_fmaf(hFr, Vn, phat);
        F[2] = hFr * V1;
        F[3] = hFr * V2;
        F[4] = __builtin_fmaf(Fr, __builtin_fmaf(cg, ibeta_ln, 0.5f * vv), 0.5f * phat * Vn);
    }

    __device__ static void diag(const Node &A, double gamma, float *F) {
        float p = 0.5f * A.r * rcpf(A.b);
        float rvn = A.r * A.vn;
        float q = A.vn * A.vn + A.vt1 * A.vt1 + A.vt2 * A.vt2;
        F[0] = rvn;
        F[1] = __builtin_fmaf(rvn, A.vn, p);
        F[2] = rvn * A.vt1;
        F[3] = rvn * A.vt2;
        F[4] = A.vn * ((float)(gamma / (gamma - 1.0)) * p + 0.5f * A.r * q);
    }

    __device__ static int out_array(int k, int m) { return EulerFP64::out_array(k, m); }
};

}  // namespace dev
}  // namespace sfhad
