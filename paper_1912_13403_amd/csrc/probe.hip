// Measurement utilities (not steps of the method): the device's sustained
// FP64 matrix-core rate and HBM copy bandwidth, measured with kernels of the
// same kind as the solve's, to set beside the published peaks of the
// roofline (78.6 TFLOP/s FP64 dense, 8 TB/s).
#include "hsdm_internal.h"

namespace {

constexpr int PROBE_ACC = 8;  // independent accumulators per wavefront

// Every wavefront runs iters rounds of PROBE_ACC independent FP64 16x16x4
// MFMAs (2048 flops each); the sum of its accumulators is stored only if it
// equals a value it cannot take, so the products are kept but nothing is
// written.
__global__ __launch_bounds__(256) void mfma_probe_kernel(int iters, double seed, double* out) {
  const int lane = threadIdx.x & 63;
  const double a = seed + lane * 1e-3, b = seed - lane * 1e-3;
  dbl4 acc[PROBE_ACC];
#pragma unroll
  for (int k = 0; k < PROBE_ACC; k++) acc[k] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int k = 0; k < PROBE_ACC; k++)
      acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < PROBE_ACC; k++) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (s == -1.0e300) out[0] = s;
}

// dst = src, 16 bytes per thread and step, grid-stride
__global__ __launch_bounds__(256) void copy_probe_kernel(const double2* src, double2* dst,
                                                         long n2) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long)gridDim.x * 256)
    dst[i] = src[i];
}

// Time of the second of two launches of `launch` on s, in ms.
template <class F>
hipError_t time_second(F launch, hipStream_t s, float& ms) {
  hipEvent_t e0, e1;
  HSDM_TRY(hipEventCreate(&e0));
  hipError_t err = hipEventCreate(&e1);
  if (err != hipSuccess) {
    (void)hipEventDestroy(e0);
    return err;
  }
  err = launch();
  if (err == hipSuccess) err = hipEventRecord(e0, s);
  if (err == hipSuccess) err = launch();
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return err;
}

int compute_units() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

}  // namespace

hipError_t probe_fp64_mfma(int iters, double* out, hipStream_t s) {
  const int cus = compute_units();
  if (cus <= 0) return hipErrorInvalidDevice;
  double* sink = nullptr;
  HSDM_TRY(hipMalloc(&sink, sizeof(double)));
  const dim3 grid(2 * cus), block(256);  // two workgroups of four wavefronts per unit
  float ms = 0.0f;
  hipError_t err = time_second(
      [&]() {
        HSDM_LAUNCH(mfma_probe_kernel, grid, block, 0, s, iters, 1.0, sink);
        return hipGetLastError();
      },
      s, ms);
  (void)hipFree(sink);
  HSDM_TRY(err);
  const double flops = (double)grid.x * (256 / 64) * (double)iters * PROBE_ACC * 2048.0;
  out[0] = flops / (ms * 1e-3) / 1e12;
  out[1] = ms;
  out[2] = flops;
  return hipSuccess;
}

hipError_t probe_hbm_copy(double bytes, double* out, hipStream_t s) {
  const int cus = compute_units();
  if (cus <= 0) return hipErrorInvalidDevice;
  const long n2 = (long)(bytes / 16.0);
  double2 *src = nullptr, *dst = nullptr;
  HSDM_TRY(hipMalloc(&src, (size_t)n2 * 16));
  hipError_t err = hipMalloc(&dst, (size_t)n2 * 16);
  if (err != hipSuccess) {
    (void)hipFree(src);
    return err;
  }
  float ms = 0.0f;  // (the contents of src do not matter to a copy)
  err = time_second(
        [&]() {
          HSDM_LAUNCH(copy_probe_kernel, dim3(8 * cus), dim3(256), 0, s, src, dst, n2);
          return hipGetLastError();
        },
        s, ms);
  (void)hipFree(src);
  (void)hipFree(dst);
  HSDM_TRY(err);
  const double moved = 2.0 * (double)n2 * 16.0;  // read and written
  out[0] = moved / (ms * 1e-3) / 1e9;
  out[1] = ms;
  out[2] = moved;
  return hipSuccess;
}
