// Device helpers with no floating-point arithmetic, shared by the kernels:
// cross-lane reads within a wavefront, the XCD-aware order of tiles, one bit
// of a bitmap.  Kept apart from the geometry header, whose file-wide
// no-contraction rule (for bit-exact tagging) must not reach the dense
// kernels.
#pragma once

#include "internal.h"

namespace ibm {

__device__ __forceinline__ bool test_bit(const uint32_t* m, int64_t n) {
  return (m[n >> 5] >> (n & 31)) & 1u;
}

// XCD-aware tile order: workgroups are dispatched round-robin over the 8
// XCDs of the chip, each with its own L2.  Block b runs on XCD b % 8; give
// XCD x the contiguous range of tiles [x T/8, (x+1) T/8) so that tiles that
// share halo rows (neighbours in x, z and the wall-normal direction) are
// processed by the same L2, close together in time.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t T) {
  const int64_t per = T / NUM_XCD, rem = T % NUM_XCD;
  const int64_t x = b % NUM_XCD, r = b / NUM_XCD;
  // XCDs 0..rem-1 own per+1 tiles, the others per tiles
  if (r < per || (r == per && x < rem)) return x * per + (x < rem ? x : rem) + r;
  return b;  // unreachable for b < T
}

// XCD band order for stencil passes over tiles (it, kt, j) of a [j][k][i]
// field on large planes: the k-tiles are cut into bands of BW, dealt to the
// XCDs round robin (XCD x takes bands x, x + 8, ...), and each XCD walks its
// band plane by plane, j slowest, before the next one.  The planes j-1, j,
// j+1 of a band are then a few hundred KB, recent in the XCD's own L2 when
// a stencil reads them again (with whole-plane slabs per XCD, a plane of
// phi at 1024 x 1024 cells is 8 MB, twice an L2, and the plane below was
// fetched from HBM again).  The grid has xcd_band_blocks() blocks; padding
// blocks get false.
__device__ __forceinline__ bool xcd_band_tile(int64_t b, int nbx, int nbz, int ny, int BW,
                                              int& it, int& kt, int& j) {
  const int x = (int)(b % NUM_XCD);
  const int64_t r = b / NUM_XCD;
  const int64_t per_band = (int64_t)nbx * BW * ny;
  const int band = x + NUM_XCD * (int)(r / per_band);
  const int64_t rem = r % per_band;
  j = (int)(rem / ((int64_t)nbx * BW));
  const int rem2 = (int)(rem % ((int64_t)nbx * BW));
  kt = band * BW + rem2 / nbx;
  it = rem2 % nbx;
  return kt < nbz;
}

// The value v of lane `src` of this wavefront (ds_bpermute: no LDS storage,
// no barrier).
__device__ __forceinline__ double lane_read(double v, int src) {
  const int a = src << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_read(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// orders this wavefront's LDS writes before its later LDS reads of other
// lanes' values
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Grouped launches (the batched form): one launch runs the blocks of several
// simulations' launches of one kernel.  The grouped instantiation of a
// kernel takes a GrpTab instead of its argument record: the records (ksize
// bytes each), the block offsets of the members (n + 1 prefix sums), each
// member's grid and a member index per block; a block reads its member (one
// load: a search over the offsets cost small blocks several dependent
// loads) and runs as that member's block (GrpTab: internal.h).  grp_enter
// gives the argument record and the block's position and grid, in both
// instantiations.
template <typename KT, bool G>
struct GArgT {
  using type = KT;
};
template <typename KT>
struct GArgT<KT, true> {
  using type = GrpTab;
};
template <typename KT, bool G>
using GArg = typename GArgT<KT, G>::type;

template <typename KT, bool G>
__device__ __forceinline__ const KT& grp_enter(const GArg<KT, G>& A, uint3& bid, uint3& gdim) {
  if constexpr (!G) {
    bid = make_uint3(blockIdx.x, blockIdx.y, blockIdx.z);
    gdim = make_uint3(gridDim.x, gridDim.y, gridDim.z);
    return A;
  } else {
    const uint32_t b = blockIdx.x;
    const int lo = __builtin_amdgcn_readfirstlane((int)A.bm[b]);
    const uint32_t l = b - A.boff[lo];
    const uint32_t gx = A.gdim[3 * lo], gy = A.gdim[3 * lo + 1], gz = A.gdim[3 * lo + 2];
    gdim = make_uint3(gx, gy, gz);
    bid = make_uint3(l % gx, (l / gx) % gy, l / (gx * gy));
    return *reinterpret_cast<const KT*>(A.k + (size_t)lo * (size_t)A.ksize);
  }
}

// Raw buffer access (gfx9 buffer descriptor, no stride, `bytes` records):
// a uniform base in the descriptor, a per-lane byte offset in a vector
// register and a uniform byte offset in a scalar register, so a loop over
// rows at a uniform stride holds one vector offset for all rows.  Offsets at
// or past `bytes` read 0 and drop stores.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t vo,
                                                 uint32_t so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, uint32_t vo,
                                       uint32_t so) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, uint32_t vo,
                                       uint32_t so) {
  typedef int i2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i2, v), r, (int)vo, (int)so, 0);
}

}  // namespace ibm
