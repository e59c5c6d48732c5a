// Diagnostic entry point: the per-node logarithm the volume kernels stage
// (step a1), evaluated on a device array so that tests can check it
// directly against a high-precision reference.
#include "kernels_common.h"
#include "sfhad_internal.h"

namespace sfhad {
namespace dev {

__global__ void __launch_bounds__(256) log1p_kernel(const double *__restrict__ x, double *__restrict__ y,
                                                    int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = log1p_series(x[i]);
}

}  // namespace dev
}  // namespace sfhad

extern "C" int sf_diag_log1p(const double *x, int64_t n, double *y, void *stream) {
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
    hipLaunchKernelGGL(sfhad::dev::log1p_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), x, y, n);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        sfhad::set_error(std::string("log1p_kernel launch: ") + hipGetErrorString(err));
        return SF_ERR_HIP;
    }
    return SF_OK;
}
