// Device build of the GPU path's per-tetrahedron arithmetic (chi0_math.h), for GPU checks of the
// device-only code (the hardware reciprocal with its third-order step, the device FP32
// logarithm, the compiler's contractions) against the oracle and the host build.  Test
// infrastructure: the product library does not use it.
#include <hip/hip_runtime.h>

#include "../../paper_1407_3444_amd/csrc/chi0_math.h"

using namespace chi0;

namespace {

// what: 0 rcp(x), 1 log_pos(x), 2 near_eval, 3 near_eval_fast (flag: entry series needed),
// 4 near_eval32, 5 tetra_weight_sum (the one-frequency far / near choice), 6 rcp(float)
__global__ void dc_kernel(int what, int n, const double *x, const double *D, const double *W, const double *om,
                          double *out, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (what == 0) { out[2 * i] = rcp(x[i]); out[2 * i + 1] = 0.0; return; }
    if (what == 1) { out[2 * i] = log_pos(x[i]); out[2 * i + 1] = 0.0; return; }
    if (what == 6) { out[2 * i] = (double)rcp((float)x[i]); out[2 * i + 1] = 0.0; return; }
    double y[4] = {D[4 * i], D[4 * i + 1], D[4 * i + 2], D[4 * i + 3]};
    double w[4] = {W[4 * i], W[4 * i + 1], W[4 * i + 2], W[4 * i + 3]};
    cplx z = cmk(0.0, 0.0);
    int f = 0;
    if (what == 5) {
        z = tetra_weight_sum(y, w, om[i]);
    } else {
        sort4(y, w);
        if (what == 2) z = near_eval(y, w, om[i]);
        if (what == 4) z = near_eval32(y, w, om[i]);
        if (what == 3) {
            bool need = false;
            z = near_eval_fast(y, w, om[i], need);
            f = need ? 1 : 0;
        }
    }
    out[2 * i] = z.re;
    out[2 * i + 1] = z.im;
    flag[i] = f;
}

}  // namespace

extern "C" {

// Evaluates case i of n on the GPU: x[i] (what 0, 1, 6) or the final tetrahedron D[i][4], W[i][4]
// at om[i]; out[i][2] = (re, im), flag[i] as above.  Host arrays; returns the HIP error code.
int dc_eval(int what, int n, const double *x, const double *D, const double *W, const double *om, double *out,
            int *flag)
{
    if (n < 1) return 0;
    double *dx = nullptr, *dD = nullptr, *dW = nullptr, *dom = nullptr, *dout = nullptr;
    int *dflag = nullptr;
    const size_t s1 = sizeof(double) * n, s4 = 4 * s1;
    hipError_t e = hipMalloc(&dx, s1);
    if (e == hipSuccess) e = hipMalloc(&dD, s4);
    if (e == hipSuccess) e = hipMalloc(&dW, s4);
    if (e == hipSuccess) e = hipMalloc(&dom, s1);
    if (e == hipSuccess) e = hipMalloc(&dout, 2 * s1);
    if (e == hipSuccess) e = hipMalloc(&dflag, sizeof(int) * n);
    if (e == hipSuccess) e = hipMemcpy(dx, x, s1, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dD, D, s4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dW, W, s4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dom, om, s1, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(dc_kernel, dim3((n + 127) / 128), dim3(128), 0, 0, what, n, dx, dD, dW, dom, dout, dflag);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, 2 * s1, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(flag, dflag, sizeof(int) * n, hipMemcpyDeviceToHost);
    hipFree(dx);
    hipFree(dD);
    hipFree(dW);
    hipFree(dom);
    hipFree(dout);
    hipFree(dflag);
    return (int)e;
}

}  // extern "C"
