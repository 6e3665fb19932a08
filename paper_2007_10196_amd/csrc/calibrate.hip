// Issue-rate calibration of the VALU (a measurement hook, not part of the method):
// each kernel runs long chains of independent operations of one instruction class,
// so that the time of a launch gives the cycles one SIMD spends per wave64
// instruction of that class.  The kernel-level issue floors quoted for the stage and
// prolongation kernels are priced with these rates.
#include "sgw_api_internal.h"

namespace {

constexpr int CAL_ITERS = 4096; // loop trips; each trip issues 8 instructions of the class (16 for INT32)

template <int OP>
__global__ void __launch_bounds__(SGW_BLOCK) cal_kernel(float* fout, double* dout, float fb, float fc, int ib)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (OP == 4) {
        double a[8];
#pragma unroll
        for (int j = 0; j < 8; j++) a[j] = gid * 1e-7 + j;
        for (int i = 0; i < CAL_ITERS; i++) {
#pragma unroll
            for (int j = 0; j < 8; j++) a[j] = fma(a[j], (double)fb, (double)fc);
        }
        double s = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) s += a[j];
        dout[gid] = s;
    } else if (OP == 3) {
        int a[8];
#pragma unroll
        for (int j = 0; j < 8; j++) a[j] = gid ^ j;
        for (int i = 0; i < CAL_ITERS; i++) {
#pragma unroll
            for (int j = 0; j < 8; j++) a[j] = (a[j] + ib) ^ a[(j + 1) & 7];
        }
        int s = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) s += a[j];
        fout[gid] = (float)s;
    } else {
        float a[8];
#pragma unroll
        for (int j = 0; j < 8; j++) a[j] = 1.0f + gid * 1e-7f + j;
        for (int i = 0; i < CAL_ITERS; i++) {
#pragma unroll
            for (int j = 0; j < 8; j++) a[j] = OP == 0 ? fmaf(a[j], fb, fc) : OP == 1 ? a[j] * fb : a[j] + fc;
        }
        float s = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) s += a[j];
        fout[gid] = s;
    }
}

} // namespace

extern "C" sgw_status sgw_calibrate_valu(int32_t op, int32_t blocks, void* out_dev, void* hip_stream,
                                         double* instructions_per_simd)
{
    if (op < 0 || op > 4 || blocks <= 0 || !out_dev || !instructions_per_simd)
        return sgw_fail(SGW_ERR_INVALID_ARG, "op %d blocks %d", op, blocks);
    hipStream_t s = (hipStream_t)hip_stream;
    float* f = (float*)out_dev;
    double* d = (double*)out_dev;
    hipError_t e = hipSuccess;
    switch (op) {
    case 0: hipLaunchKernelGGL(cal_kernel<0>, dim3(blocks), dim3(SGW_BLOCK), 0, s, f, d, 0.999f, 1e-3f, 7); break;
    case 1: hipLaunchKernelGGL(cal_kernel<1>, dim3(blocks), dim3(SGW_BLOCK), 0, s, f, d, 0.9999f, 1e-3f, 7); break;
    case 2: hipLaunchKernelGGL(cal_kernel<2>, dim3(blocks), dim3(SGW_BLOCK), 0, s, f, d, 0.999f, 1e-3f, 7); break;
    case 3: hipLaunchKernelGGL(cal_kernel<3>, dim3(blocks), dim3(SGW_BLOCK), 0, s, f, d, 0.999f, 1e-3f, 7); break;
    default: hipLaunchKernelGGL(cal_kernel<4>, dim3(blocks), dim3(SGW_BLOCK), 0, s, f, d, 0.999f, 1e-3f, 7); break;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return sgw_hip_fail(e, "calibration launch");
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    const double per_trip = op == 3 ? 16.0 : 8.0;
    *instructions_per_simd = (double)blocks * (SGW_BLOCK / 64) * CAL_ITERS * per_trip / (4.0 * cus);
    return SGW_OK;
}
