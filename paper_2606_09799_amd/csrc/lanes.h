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

// XCD slab order for stencil sweeps over tiles (it, kt, j) of a
// [j][k][i] field: XCD x (the blocks b with b % 8 == x) owns the band of
// k-tiles [x nbz/8, (x+1) nbz/8) and walks it plane by plane, j slowest, so
// the planes j-1, j, j+1 that a stencil touches are all recent in its own
// L2 (a band of whole planes per XCD would need three planes of every field
// at once, more than one L2 holds).  The grid has xcd_slab_blocks() blocks;
// the padding blocks of XCDs with a narrower band get false.
__device__ __forceinline__ bool xcd_slab_tile(int64_t b, int nbx, int nbz, int ny, int& it,
                                              int& kt, int& j) {
  const int x = (int)(b % NUM_XCD);
  const int64_t r = b / NUM_XCD;
  const int kt0 = (int)((int64_t)x * nbz / NUM_XCD);
  const int kt1 = (int)((int64_t)(x + 1) * nbz / NUM_XCD);
  const int64_t per_plane = (int64_t)nbx * (kt1 - kt0);
  if (per_plane == 0 || r >= per_plane * ny) return false;
  j = (int)(r / per_plane);
  const int rem = (int)(r % per_plane);
  kt = kt0 + rem / nbx;
  it = rem % nbx;
  return true;
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

}  // namespace ibm
