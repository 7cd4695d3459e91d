// Fill kernels (used instead of hipMemsetAsync so that a captured graph never
// holds memset nodes).
#include "lanes.h"

namespace ibm {

template <typename T>
struct FillK {
  T* p;
  int64_t n;
  T val;
};

template <typename T, bool G = false>
__global__ void k_fill(GArg<FillK<T>, G> grp_arg_) {
  uint3 bid, gdim;
  const FillK<T>& a = grp_enter<FillK<T>, G>(grp_arg_, bid, gdim);
  for (int64_t i = (int64_t)bid.x * blockDim.x + threadIdx.x; i < a.n;
       i += (int64_t)gdim.x * blockDim.x)
    a.p[i] = a.val;
}

template <typename T>
static void fill(Prof* pf, hipStream_t s, T* p, int64_t n, T val, const char* name) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  const FillK<T> a{p, n, val};
  IBM_LAUNCH_G(pf, name, s, (&k_fill<T, true>), dim3((unsigned)blocks), dim3(256), 0, a,
               k_fill<T><<<(int)blocks, 256, 0, s>>>(a));
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
