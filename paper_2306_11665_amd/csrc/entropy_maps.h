// Pointwise maps between the conserved variables u = (rho, rho vel, E) of 3D
// Euler and the entropy variables v = dU/du of U = -rho s/(gamma - 1),
// s = ln p - gamma ln rho:
//     v = ((gamma - s)/(gamma - 1) - rho |vel|^2/(2p), rho vel/p, -rho/p),
// and back from rho/p = -v_4: vel = v_1..3/(rho/p),
// s = gamma - (gamma - 1)(v_0 + (rho/p)|vel|^2/2),
// rho = exp((s + ln(rho/p))/(1 - gamma)), p = rho/(rho/p).
// Quotients are products with a refined reciprocal; the logarithms and the
// exponential are this library's own (log_pos, exp_fine: about one ulp, a
// third of the device library's FP64 instruction count).  Shared by the
// pointwise map kernel, the entropy-projected trace and the basis
// transformation's fused epilogue, so that all give the same bits.
#pragma once

#include "kernels_common.h"

namespace sfhad {
namespace dev {

// x: conserved, y: entropy variables; igm1 = 1/(gamma - 1)
__device__ __forceinline__ void entropy_from_conserved(const double (&x)[5], double g, double igm1,
                                                       double (&y)[5]) {
    const double irho = rcp_fine(x[0]);
    const double vx = x[1] * irho, vy = x[2] * irho, vz = x[3] * irho;
    const double q = vx * vx + vy * vy + vz * vz;
    const double p = (g - 1.0) * (x[4] - 0.5 * x[0] * q);
    const double rp = x[0] * rcp_fine(p);
    const double s = log_pos(p) - g * log_pos(x[0]);
    y[0] = (g - s) * igm1 - 0.5 * rp * q;
    y[1] = rp * vx;
    y[2] = rp * vy;
    y[3] = rp * vz;
    y[4] = -rp;
}

// x: entropy variables, y: conserved
__device__ __forceinline__ void conserved_from_entropy(const double (&x)[5], double g, double igm1,
                                                       double (&y)[5]) {
    const double rp = -x[4];
    const double irp = rcp_fine(rp);
    const double vx = x[1] * irp, vy = x[2] * irp, vz = x[3] * irp;
    const double q = vx * vx + vy * vy + vz * vz;
    const double s = g - (g - 1.0) * (x[0] + 0.5 * rp * q);
    const double rho = exp_fine(-(s + log_pos(rp)) * igm1);
    const double p = rho * irp;
    y[0] = rho;
    y[1] = rho * vx;
    y[2] = rho * vy;
    y[3] = rho * vz;
    y[4] = p * igm1 + 0.5 * rho * q;
}

}  // namespace dev
}  // namespace sfhad
