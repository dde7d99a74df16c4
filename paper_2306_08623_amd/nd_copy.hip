// nd_copy -- a plain device-to-device copy kernel of known size, used to
// calibrate hardware byte counters (FETCH_SIZE / WRITE_SIZE) against a
// kernel that reads and writes exactly `bytes` bytes once each.
//
//   nd_copy <bytes> [launches]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

__global__ void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

int main(int argc, char **argv) {
  const size_t bytes = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : (1ull << 30);
  const int launches = argc > 2 ? std::atoi(argv[2]) : 3;
  const size_t n = bytes / sizeof(uint4);
  uint4 *a = nullptr, *b = nullptr;
  if (n == 0 || hipMalloc(&a, n * sizeof(uint4)) != hipSuccess ||
      hipMalloc(&b, n * sizeof(uint4)) != hipSuccess) {
    std::fprintf(stderr, "allocation of 2 x %zu bytes failed\n", n * sizeof(uint4));
    return 1;
  }
  if (hipMemset(a, 1, n * sizeof(uint4)) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  for (int i = 0; i < launches; i++) {
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, nullptr, a, b, n);
    (void)hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess) return 1;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    std::printf("launch %d: copied %zu bytes (read %zu + write %zu) in %.3f ms = %.1f GB/s\n", i,
                n * sizeof(uint4), n * sizeof(uint4), n * sizeof(uint4), ms,
                2.0 * n * sizeof(uint4) / (ms * 1e6));
  }
  (void)hipFree(a);
  (void)hipFree(b);
  return 0;
}
