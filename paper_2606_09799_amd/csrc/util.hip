// Fill kernels (used instead of hipMemsetAsync so that a captured graph never
// holds memset nodes).
#include "internal.h"

namespace ibm {

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

template <typename T>
static void fill(Prof* pf, hipStream_t s, T* p, int64_t n, T val, const char* name) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  IBM_LAUNCH(pf, name, s, k_fill<T><<<(int)blocks, 256, 0, s>>>(p, n, val));
}

void launch_fill_u32(Prof* pf, hipStream_t s, uint32_t* p, int64_t n, uint32_t val) {
  fill(pf, s, p, n, val, "fill_u32");
}
void launch_fill_u8(Prof* pf, hipStream_t s, uint8_t* p, int64_t n, uint8_t val) {
  fill(pf, s, p, n, val, "fill_u8");
}
void launch_fill_u64(Prof* pf, hipStream_t s, u64* p, int64_t n, u64 val) {
  fill(pf, s, p, n, val, "fill_u64");
}
void launch_fill_i32(Prof* pf, hipStream_t s, int32_t* p, int64_t n, int32_t val) {
  fill(pf, s, p, n, val, "fill_i32");
}
void launch_fill_f64(Prof* pf, hipStream_t s, double* p, int64_t n, double val) {
  fill(pf, s, p, n, val, "fill_f64");
}

}  // namespace ibm
