// Tagging of the three staggered lattices (paper Alg. 1, Sec. 3.1) and of
// the boundary cells C_B (Sec. 3.2).
//
// Pipeline, all on the device and free of host synchronisation:
//   1. k_tag_pairs, pass 0: one 64-lane wavefront per (triangle, lattice)
//      visits the nodes of the triangle's inflated bounding box, computes the
//      closest point X, N = x - X and the six-neighbour sign test; every
//      classifying pair lowers best_d[node] (the bit pattern of |N|^2, an
//      order-preserving key for non-negative doubles) with an integer
//      atomicMin and sets the node's mask bit.
//   2. pass 1: the same pairs; those whose |N|^2 equals best_d[node] lower
//      best_t[node] with atomicMin on the triangle id.  Both passes are
//      order-independent, so the result is deterministic.
//   3. Compaction of each bitmap (block popcounts, one scan, emission in
//      increasing node order): the sorted forcing list, its triangles, and a
//      sparse reset of best_d / best_t for the next call.
//   4. C_B from the u list (all six faces forcing), compacted the same way.
#pragma clang fp contract(off)

#include "geom.h"

namespace ibm {

struct TagK {
  GridView g;
  const BodyDev* bodies;
  int nbody, ntri, pass;
  uint32_t* mask[3];
  u64* best_d[3];
  int32_t* best_t[3];
  uint32_t* flags;
};

__global__ __launch_bounds__(64) void k_tag_pairs(TagK a) {
  const int t = blockIdx.x;
  const int c = blockIdx.y;
  if (t >= a.ntri) return;
  const GridView& g = a.g;
  double A[3], B[3], C[3];
  const double* vel;
  int vid[3];
  load_triangle(a.bodies, a.nbody, t, A, B, C, &vel, vid);
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = fmin(A[d], fmin(B[d], C[d]));
    hi[d] = fmax(A[d], fmax(B[d], C[d]));
  }
  const Lattice L = lattice(g, c);
  const Box bx = candidate_box(g, L, lo, hi);
  const int ni = bx.i1 - bx.i0 + 1, ne = bx.e1 - bx.e0 + 1, nk = bx.k1 - bx.k0 + 1;
  if (ni + 1 >= g.nx || nk + 1 >= g.nz) {  // a node would have two images
    if (threadIdx.x == 0) atomicOr(a.flags, FLAG_GEOM);
    return;
  }
  const int64_t total = (int64_t)ni * ne * nk;
  uint32_t* mask = a.mask[c];
  u64* best_d = a.best_d[c];
  int32_t* best_t = a.best_t[c];
  for (int64_t q = threadIdx.x; q < total; q += blockDim.x) {
    const int ii = bx.i0 + (int)(q % ni);
    const int64_t r = q / ni;
    const int ee = bx.e0 + (int)(r % ne);
    const int kk = bx.k0 + (int)(r / ne);
    const double p[3] = {((double)ii + L.ox) * g.dx, L.ext[ee], ((double)kk + L.oz) * g.dz};
    const ClosestPt X = closest_point(p, A, B, C);
    const double N0 = p[0] - X.x[0], N1 = p[1] - X.x[1], N2 = p[2] - X.x[2];
    const double n2 = dot3(N0, N1, N2, N0, N1, N2);
    bool f = (n2 == 0.0);
    if (!f) {
      // the six same-lattice neighbours x_n; (x_n - X) . N < 0 classifies
      const double xm = ((double)(ii - 1) + L.ox) * g.dx;
      const double xp = ((double)(ii + 1) + L.ox) * g.dx;
      const double zm = ((double)(kk - 1) + L.oz) * g.dz;
      const double zp = ((double)(kk + 1) + L.oz) * g.dz;
      const double ym = L.ext[ee - 1], yp = L.ext[ee + 1];
      f = dot3(xm - X.x[0], N1, N2, N0, N1, N2) < 0.0 ||
          dot3(xp - X.x[0], N1, N2, N0, N1, N2) < 0.0 ||
          dot3(N0, ym - X.x[1], N2, N0, N1, N2) < 0.0 ||
          dot3(N0, yp - X.x[1], N2, N0, N1, N2) < 0.0 ||
          dot3(N0, N1, zm - X.x[2], N0, N1, N2) < 0.0 ||
          dot3(N0, N1, zp - X.x[2], N0, N1, N2) < 0.0;
    }
    if (!f) continue;
    const int j = (c == 1) ? ee : ee - 1;
    const int64_t node = ((int64_t)j * g.nz + wrapi(kk, g.nz)) * g.nx + wrapi(ii, g.nx);
    const u64 bits = (u64)__double_as_longlong(n2);
    if (a.pass == 0) {
      atomicMin(&best_d[node], bits);
      atomicOr(&mask[node >> 5], 1u << (node & 31));
    } else if (best_d[node] == bits) {
      atomicMin(&best_t[node], t);
    }
  }
}

// ------------------------------------------------------------ compaction
constexpr int CT = 256;       // threads per block
constexpr int CWT = 4;        // mask words per thread
constexpr int CWB = CT * CWT; // mask words per block

__device__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < CT; off <<= 1) {
    int64_t add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int64_t incl = sh[t];
  *total = sh[CT - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(CT) void k_count(const uint32_t* __restrict__ mask, int64_t nwords,
                                              int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[CT];
  const int64_t base = (int64_t)blockIdx.x * CWB + (int64_t)threadIdx.x * CWT;
  int64_t c = 0;
  for (int q = 0; q < CWT; ++q)
    if (base + q < nwords) c += __popc(mask[base + q]);
  int64_t tot;
  block_excl_scan(c, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of nb block sums in place (one block); total -> *count
__global__ __launch_bounds__(1024) void k_scan(int64_t* __restrict__ bsum, int64_t nb,
                                               int64_t* __restrict__ count) {
  __shared__ int64_t sh[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (nb + 1023) / 1024;
  const int64_t lo = t * chunk, hi = (lo + chunk < nb) ? lo + chunk : nb;
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += bsum[i];
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  int64_t run = sh[t] - s;
  for (int64_t i = lo; i < hi; ++i) {
    int64_t v = bsum[i];
    bsum[i] = run;
    run += v;
  }
  if (t == 1023) *count = sh[1023];
}

__global__ __launch_bounds__(CT) void k_emit(const uint32_t* __restrict__ mask, int64_t nwords,
                                             const int64_t* __restrict__ boff,
                                             int64_t* __restrict__ idx, int32_t* __restrict__ tri,
                                             u64* __restrict__ best_d, int32_t* __restrict__ best_t,
                                             int64_t cap, uint32_t* flags) {
  __shared__ int64_t sh[CT];
  const int64_t base = (int64_t)blockIdx.x * CWB + (int64_t)threadIdx.x * CWT;
  uint32_t w[CWT];
  int64_t c = 0;
  for (int q = 0; q < CWT; ++q) {
    w[q] = (base + q < nwords) ? mask[base + q] : 0u;
    c += __popc(w[q]);
  }
  int64_t tot;
  int64_t pos = boff[blockIdx.x] + block_excl_scan(c, sh, &tot);
  bool over = false;
  for (int q = 0; q < CWT; ++q) {
    uint32_t m = w[q];
    while (m) {
      const int b = __ffs(m) - 1;
      m &= m - 1;
      const int64_t node = (base + q) * 32 + b;
      if (pos < cap) {
        idx[pos] = node;
        if (tri) tri[pos] = best_t[node];
      } else {
        over = true;
      }
      if (best_d) {
        best_d[node] = ~0ull;
        best_t[node] = 0x7fffffff;
      }
      ++pos;
    }
  }
  if (over) atomicOr(flags, FLAG_CAPACITY);
}

// C_B: cells all six of whose faces carry forcing nodes (checked from the
// u list: the west face u(i,j,k) of cell (i,j,k)).
__global__ void k_cells(GridView g, const int64_t* __restrict__ idx_u,
                        const int64_t* __restrict__ count, int64_t cap,
                        const uint32_t* __restrict__ mu, const uint32_t* __restrict__ mv,
                        const uint32_t* __restrict__ mw, uint32_t* __restrict__ cb_mask) {
  int64_t n = count[0];
  if (n > cap) n = cap;
  const int64_t plane = (int64_t)g.nz * g.nx;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = idx_u[f];
    const int i = (int)(node % g.nx);
    const int k = (int)((node / g.nx) % g.nz);
    const int64_t j = node / plane;
    const int64_t row = j * plane + (int64_t)k * g.nx;
    const int ip = (i + 1 == g.nx) ? 0 : i + 1;
    const int kp = (k + 1 == g.nz) ? 0 : k + 1;
    if (test_bit(mu, row + ip) && test_bit(mv, node) && test_bit(mv, node + plane) &&
        test_bit(mw, node) && test_bit(mw, j * plane + (int64_t)kp * g.nx + i))
      atomicOr(&cb_mask[node >> 5], 1u << (node & 31));
  }
}

static void compact(Prof* pf, hipStream_t s, const uint32_t* mask, int64_t nwords,
                    int64_t* bsum, int64_t* count_slot, int64_t* idx, int32_t* tri, u64* best_d,
                    int32_t* best_t, int64_t cap, uint32_t* flags) {
  const int64_t nb = (nwords + CWB - 1) / CWB;
  IBM_LAUNCH(pf, "tag_count", s, k_count<<<(int)nb, CT, 0, s>>>(mask, nwords, bsum));
  IBM_LAUNCH(pf, "tag_scan", s, k_scan<<<1, 1024, 0, s>>>(bsum, nb, count_slot));
  IBM_LAUNCH(pf, "tag_emit", s,
             k_emit<<<(int)nb, CT, 0, s>>>(mask, nwords, bsum, idx, tri, best_d, best_t, cap,
                                           flags));
}

void launch_tag(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nbody,
                int ntri, TagBuffers& tb, uint32_t* flags) {
  for (int c = 0; c < 3; ++c) {
    launch_fill_u32(pf, s, tb.mask[c], tb.nwords[c], 0u);
  }
  launch_fill_u32(pf, s, tb.cb_mask, tb.nwords_cb, 0u);
  if (ntri > 0) {
    TagK a;
    a.g = g;
    a.bodies = bodies;
    a.nbody = nbody;
    a.ntri = ntri;
    for (int c = 0; c < 3; ++c) {
      a.mask[c] = tb.mask[c];
      a.best_d[c] = tb.best_d[c];
      a.best_t[c] = tb.best_t[c];
    }
    a.flags = flags;
    dim3 grid(ntri, 3);
    a.pass = 0;
    IBM_LAUNCH(pf, "tag_pairs", s, k_tag_pairs<<<grid, 64, 0, s>>>(a));
    a.pass = 1;
    IBM_LAUNCH(pf, "tag_pairs", s, k_tag_pairs<<<grid, 64, 0, s>>>(a));
  }
  // the block-sum scratch is reused; kernels on one stream run in order
  for (int c = 0; c < 3; ++c)
    compact(pf, s, tb.mask[c], tb.nwords[c], tb.block_sums, tb.count + c, tb.idx[c], tb.tri[c],
            tb.best_d[c], tb.best_t[c], tb.cap, flags);
  IBM_LAUNCH(pf, "tag_cells", s,
             k_cells<<<1024, 256, 0, s>>>(g, tb.idx[0], tb.count, tb.cap, tb.mask[0], tb.mask[1],
                                          tb.mask[2], tb.cb_mask));
  compact(pf, s, tb.cb_mask, tb.nwords_cb, tb.block_sums, tb.count + 3, tb.cb, nullptr, nullptr,
          nullptr, tb.cap, flags);
}

}  // namespace ibm
