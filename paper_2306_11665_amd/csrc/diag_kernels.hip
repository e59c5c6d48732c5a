// Diagnostic entry points: the per-node logarithm the volume kernels stage
// (step a1) and the logarithm and exponential of the entropy-variable maps,
// evaluated on a device array so that tests can check them directly against
// a high-precision reference.
#include "kernels_common.h"
#include "sfhad_internal.h"

namespace sfhad {
namespace dev {

enum DiagFn { kDiagLog1p = 0, kDiagLog = 1, kDiagExp = 2 };

template <int FN>
__global__ void __launch_bounds__(256) diag_kernel(const double *__restrict__ x, double *__restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = FN == kDiagLog1p ? log1p_series(x[i]) : FN == kDiagLog ? log_pos(x[i]) : exp_fine(x[i]);
}

}  // namespace dev
}  // namespace sfhad

namespace {
template <int FN>
int diag_launch(const double *x, int64_t n, double *y, void *stream) {
    if (n < 0) {
        sfhad::set_error("n must be >= 0");
        return SF_ERR_ARG;
    }
    if (n == 0) return SF_OK;
    if (!x || !y) {
        sfhad::set_error("null x or y");
        return SF_ERR_ARG;
    }
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffLL) {
        sfhad::set_error("n too large");
        return SF_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL(sfhad::dev::diag_kernel<FN>, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), x, y, n);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        sfhad::set_error(std::string("diag_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}
}  // namespace

extern "C" int sf_diag_log1p(const double *x, int64_t n, double *y, void *stream) {
    return diag_launch<sfhad::dev::kDiagLog1p>(x, n, y, stream);
}

extern "C" int sf_diag_log(const double *x, int64_t n, double *y, void *stream) {
    return diag_launch<sfhad::dev::kDiagLog>(x, n, y, stream);
}

extern "C" int sf_diag_exp(const double *x, int64_t n, double *y, void *stream) {
    return diag_launch<sfhad::dev::kDiagExp>(x, n, y, stream);
}
