// Tagging of the three staggered lattices (paper Alg. 1, Sec. 3.1) and of
// the boundary cells C_B (Sec. 3.2).
//
// Pipeline, all on the device and free of host synchronisation:
//   1. k_tag_pairs, pass 0: one 64-lane wavefront per (triangle, lattice)
//      visits the nodes of the triangle's inflated bounding box that lie
//      within the largest neighbour spacing of its bounding box and of its
//      plane (the others cannot classify), computes the
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
  double dt;  // > 0: check the vertex displacement over dt (pass 0)
  uint32_t* mask[3];
  u64* best_d[3];
  int32_t* best_t[3];
  uint32_t* flags;
};

// Counts over an ascending array by the 64 lanes of a wavefront together
// (every lane reads the entries lane, lane + 64, ...; the counts are sums of
// ballots): one memory round trip per 64 entries instead of one per
// bisection step, and two bounds from the same reads.  lt: entries below v0
// (the lower bound of v0, numpy searchsorted side 'left'); le: entries at
// most v1 (the upper bound of v1, side 'right').
__device__ __forceinline__ void wave_bounds(const double* ext, int n, double v0, double v1,
                                            int lane, int& lt, int& le) {
  lt = 0;
  le = 0;
  for (int m = 0; m < n; m += 64) {
    const double x = (m + lane < n) ? ext[m + lane] : 0.0;
    const bool in = m + lane < n;
    lt += __popcll((u64)__ballot(in && x < v0));
    le += __popcll((u64)__ballot(in && x <= v1));
  }
}

// find_body by the lanes of a wavefront: the last body whose first triangle
// id is at most t (the ids ascend)
__device__ __forceinline__ int wave_find_body(const BodyDev* b, int nbody, int t, int lane) {
  int cnt = 0;
  for (int m = 0; m < nbody; m += 64)
    cnt += __popcll((u64)__ballot(m + lane < nbody && b[m + lane].toff <= t));
  return cnt > 0 ? cnt - 1 : 0;
}

// One wavefront per (triangle, lattice), four triangles per block (no block
// barrier: each wavefront works alone).
constexpr int TAG_TPB = 4;
template <bool G = false>
__global__ __launch_bounds__(64 * TAG_TPB) void k_tag_pairs(GArg<TagK, G> grp_arg_) {
  uint3 bid, gdim;
  const TagK& a = grp_enter<TagK, G>(grp_arg_, bid, gdim);
  (void)gdim;
  const int lane = (int)(threadIdx.x & 63);
  const int t = (int)bid.x * TAG_TPB + (int)(threadIdx.x >> 6);
  const int c = bid.y;
  if (t >= a.ntri) return;
  const GridView& g = a.g;
  double A[3], B[3], C[3];
  const double* vel;
  int vid[3];
  {
    const BodyDev& bd = a.bodies[wave_find_body(a.bodies, a.nbody, t, lane)];
    const int lt = t - bd.toff;
    vid[0] = bd.tri[3 * lt];
    vid[1] = bd.tri[3 * lt + 1];
    vid[2] = bd.tri[3 * lt + 2];
    for (int d = 0; d < 3; ++d) {
      A[d] = bd.xyz[3 * vid[0] + d];
      B[d] = bd.xyz[3 * vid[1] + d];
      C[d] = bd.xyz[3 * vid[2] + d];
    }
    vel = bd.vel;
  }
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = fmin(A[d], fmin(B[d], C[d]));
    hi[d] = fmax(A[d], fmax(B[d], C[d]));
  }
  // the one-layer fresh-cell assumption (Sec. 3.1): over dt no vertex may
  // move more than half the local spacing along an axis (the y spacing of the
  // cell the vertex lies in)
  if (a.dt > 0.0 && a.pass == 0 && c == 0) {
    bool over = false;
    for (int q = 0; q < 3; ++q) {
      const double* U = vel + 3 * vid[q];
      const double y = (q == 0) ? A[1] : (q == 1 ? B[1] : C[1]);
      int below, upto;
      wave_bounds(g.yf, g.ny + 1, y, y, lane, below, upto);
      int j = upto - 1;  // the face at or below y
      j = j < 0 ? 0 : (j > g.ny - 1 ? g.ny - 1 : j);
      over = over || fabs(U[0]) * a.dt > 0.5 * g.dx || fabs(U[2]) * a.dt > 0.5 * g.dz ||
             fabs(U[1]) * a.dt > 0.5 * g.dy[j];
    }
    if (over && lane == 0) atomicOr(a.flags, FLAG_CFL);
  }
  const Lattice L = lattice(g, c);
  // the candidate box of candidate_box, its y range counted by the lanes
  // together (the same bounds as its bisections)
  Box bx;
  {
    const double dm = g.dmax;
    bx.i0 = (int)floor((lo[0] - dm) / g.dx - L.ox) - 1;
    bx.i1 = (int)floor((hi[0] + dm) / g.dx - L.ox) + 1;
    bx.k0 = (int)floor((lo[2] - dm) / g.dz - L.oz) - 1;
    bx.k1 = (int)floor((hi[2] + dm) / g.dz - L.oz) + 1;
    int lb, ub;
    wave_bounds(L.ext, L.next, lo[1] - dm, hi[1] + dm, lane, lb, ub);
    const int e0 = lb - 1, e1 = ub;
    bx.e0 = e0 < L.e_first ? L.e_first : (e0 > L.e_last ? L.e_last : e0);
    bx.e1 = e1 < L.e_first ? L.e_first : (e1 > L.e_last ? L.e_last : e1);
  }
  const int ni = bx.i1 - bx.i0 + 1, nk = bx.k1 - bx.k0 + 1;
  if (ni + 1 >= g.nx || nk + 1 >= g.nz) {  // a node would have two images
    if (lane == 0) atomicOr(a.flags, FLAG_GEOM);
    return;
  }
  // The nodes scanned: those of the box within the largest neighbour spacing
  // (plus a relative margin of 1e-6, beyond the prune's below) of the
  // triangle's bounding box along each axis; the box's margin nodes and the
  // rest cannot classify (see the prune below).
  const double dms = g.dmax * (1.0 + 1e-6);
  const int si0 = max(bx.i0, (int)floor((lo[0] - dms) / g.dx - L.ox));
  const int si1 = min(bx.i1, (int)ceil((hi[0] + dms) / g.dx - L.ox));
  const int sk0 = max(bx.k0, (int)floor((lo[2] - dms) / g.dz - L.oz));
  const int sk1 = min(bx.k1, (int)ceil((hi[2] + dms) / g.dz - L.oz));
  int slb, sub;
  wave_bounds(L.ext, L.next, lo[1] - dms, hi[1] + dms, lane, slb, sub);
  const int se0 = max(bx.e0, slb);
  const int se1 = min(bx.e1, sub - 1);
  const int sni = si1 - si0 + 1, sne = se1 - se0 + 1, snk = sk1 - sk0 + 1;
  // (the scanned box lies within the candidate box, whose extents are below
  // the periodic lengths and ny + 2: the node index fits 32 bits)
  const int total = (sni > 0 && sne > 0 && snk > 0) ? sni * sne * snk : 0;
  uint32_t* mask = a.mask[c];
  u64* best_d = a.best_d[c];
  int32_t* best_t = a.best_t[c];
  auto node_pos = [&](int q, int& ii, int& ee, int& kk, double p[3]) {
    ii = si0 + q % sni;
    const int r = q / sni;
    ee = se0 + r % sne;
    kk = sk0 + r / sne;
    p[0] = ((double)ii + L.ox) * g.dx;
    p[1] = L.ext[ee];
    p[2] = ((double)kk + L.oz) * g.dz;
  };
  auto visit = [&](int q) {
    int ii, ee, kk;
    double p[3];
    node_pos(q, ii, ee, kk, p);
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
    if (!f) return;
    const int j = (c == 1) ? ee : ee - 1;
    const int64_t node = ((int64_t)j * g.nz + wrapi(kk, g.nz)) * g.nx + wrapi(ii, g.nx);
    const u64 bits = (u64)__double_as_longlong(n2);
    if (a.pass == 0) {
      atomicMin(&best_d[node], bits);
      atomicOr(&mask[node >> 5], 1u << (node & 31));
    } else if (best_d[node] == bits) {
      atomicMin(&best_t[node], t);
    }
  };
  // Conservative prune.  A node classifies only if some neighbour x_n gives
  // (x_n - X).N < 0, i.e. |N|^2 < (x - x_n).N <= h |N| with h the spacing to
  // that neighbour (at most dmax), or if N = 0: |N| < dmax either way (up to
  // the rounding of the computed test, relative 1e-15, far inside the margin
  // below).  |N| = |x - X| is at least the distance of x to the triangle's
  // bounding box and to its plane, so a node for which either exceeds dmax
  // (with the margin) cannot classify and is skipped; the classification
  // itself is unchanged.  A degenerate triangle has a NaN plane distance,
  // which prunes nothing.  The surviving nodes are queued per wavefront in
  // LDS (ballot and lane prefix count) and visited 64 at a time, so that the
  // lanes of a visit are all busy.
  const double e1x = B[0] - A[0], e1y = B[1] - A[1], e1z = B[2] - A[2];
  const double e2x = C[0] - A[0], e2y = C[1] - A[1], e2z = C[2] - A[2];
  const double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
  const double cn = sqrt(dot3(cx, cy, cz, cx, cy, cz));
  const double un0 = cx / cn, un1 = cy / cn, un2 = cz / cn;
  const double lim = g.dmax * g.dmax * (1.0 + 1e-6);
  __shared__ int qbuf[TAG_TPB][128];
  int* qb = qbuf[threadIdx.x >> 6];
  int cnt = 0;  // queued nodes (uniform over the wavefront, below 64 between visits)
  for (int base = 0; base < total; base += 64) {
    const int q = base + lane;
    bool cand = false;
    if (q < total) {
      int ii, ee, kk;
      double p[3];
      node_pos(q, ii, ee, kk, p);
      const double b0 = fmax(fmax(lo[0] - p[0], p[0] - hi[0]), 0.0);
      const double b1 = fmax(fmax(lo[1] - p[1], p[1] - hi[1]), 0.0);
      const double b2 = fmax(fmax(lo[2] - p[2], p[2] - hi[2]), 0.0);
      const double pd = dot3(p[0] - A[0], p[1] - A[1], p[2] - A[2], un0, un1, un2);
      cand = !(dot3(b0, b1, b2, b0, b1, b2) > lim) && !(pd * pd > lim);
    }
    const u64 bal = (u64)__ballot(cand);
    if (cand) {
      const int below = (int)__builtin_amdgcn_mbcnt_hi(
          (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      qb[cnt + below] = q;
    }
    cnt += __popcll(bal);
    if (cnt >= 64) {
      wave_sync();
      const int qq = qb[lane];
      const int rem = cnt - 64;
      const int mv = (lane < rem) ? qb[64 + lane] : 0;
      wave_sync();
      if (lane < rem) qb[lane] = mv;
      cnt = rem;
      visit(qq);
    }
  }
  if (cnt > 0) {
    wave_sync();
    if (lane < cnt) visit(qb[lane]);
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

// Up to three lists compacted by one launch of each kernel: list y of the
// grid (blockIdx.y) with its own mask, block sums, outputs and count.
struct CompactSet {
  const uint32_t* mask[3];
  int64_t nwords[3];
  int64_t nb[3];        // blocks of CWB words
  int64_t* bsum[3];
  int64_t* idx[3];
  int32_t* tri[3];      // forcing triangles (NULL for C_B)
  u64* best_d[3];       // reset to the empty key after reading (NULL for C_B)
  int32_t* best_t[3];
  int64_t* count[3];
  int64_t cap;
  uint32_t* flags;
};

template <bool G = false>
__global__ __launch_bounds__(CT) void k_count(GArg<CompactSet, G> grp_arg_) {
  uint3 bid, gdim;
  const CompactSet& S = grp_enter<CompactSet, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  __shared__ int64_t sh[CT];
  const int l = bid.y;
  if ((int64_t)bid.x >= S.nb[l]) return;  // block-uniform
  const uint32_t* mask = S.mask[l];
  const int64_t nwords = S.nwords[l];
  const int64_t base = (int64_t)bid.x * CWB + (int64_t)threadIdx.x * CWT;
  int64_t c = 0;
  for (int q = 0; q < CWT; ++q)
    if (base + q < nwords) c += __popc(mask[base + q]);
  int64_t tot;
  block_excl_scan(c, sh, &tot);
  if (threadIdx.x == 0) S.bsum[l][bid.x] = tot;
}

// exclusive scan of a list's nb block sums in place (one block per list);
// total -> its count
template <bool G = false>
__global__ __launch_bounds__(1024) void k_scan(GArg<CompactSet, G> grp_arg_) {
  uint3 bid, gdim;
  const CompactSet& S = grp_enter<CompactSet, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  __shared__ int64_t sh[1024];
  const int l = bid.x;
  int64_t* bsum = S.bsum[l];
  const int64_t nb = S.nb[l];
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
  if (t == 1023) *S.count[l] = sh[1023];
}

template <bool G = false>
__global__ __launch_bounds__(CT) void k_emit(GArg<CompactSet, G> grp_arg_) {
  uint3 bid, gdim;
  const CompactSet& S = grp_enter<CompactSet, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  __shared__ int64_t sh[CT];
  const int l = bid.y;
  if ((int64_t)bid.x >= S.nb[l]) return;  // block-uniform
  const uint32_t* mask = S.mask[l];
  const int64_t nwords = S.nwords[l];
  int64_t* idx = S.idx[l];
  int32_t* tri = S.tri[l];
  u64* best_d = S.best_d[l];
  int32_t* best_t = S.best_t[l];
  const int64_t cap = S.cap;
  const int64_t base = (int64_t)bid.x * CWB + (int64_t)threadIdx.x * CWT;
  uint32_t w[CWT];
  int64_t c = 0;
  for (int q = 0; q < CWT; ++q) {
    w[q] = (base + q < nwords) ? mask[base + q] : 0u;
    c += __popc(w[q]);
  }
  int64_t tot;
  int64_t pos = S.bsum[l][bid.x] + block_excl_scan(c, sh, &tot);
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
  if (over) atomicOr(S.flags, FLAG_CAPACITY);
}

// zero up to four bitmaps in one launch (array blockIdx.y)
struct ZeroMasksK {
  uint32_t* m0;
  int64_t n0;
  uint32_t* m1;
  int64_t n1;
  uint32_t* m2;
  int64_t n2;
  uint32_t* m3;
  int64_t n3;
};
template <bool G = false>
__global__ __launch_bounds__(256) void k_zero_masks(GArg<ZeroMasksK, G> grp_arg_) {
  uint3 bid, gdim;
  const ZeroMasksK& P_ = grp_enter<ZeroMasksK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  uint32_t* m0 = P_.m0;
  int64_t n0 = P_.n0;
  uint32_t* m1 = P_.m1;
  int64_t n1 = P_.n1;
  uint32_t* m2 = P_.m2;
  int64_t n2 = P_.n2;
  uint32_t* m3 = P_.m3;
  int64_t n3 = P_.n3;
  uint32_t* m = bid.y == 0 ? m0 : (bid.y == 1 ? m1 : (bid.y == 2 ? m2 : m3));
  const int64_t n = bid.y == 0 ? n0 : (bid.y == 1 ? n1 : (bid.y == 2 ? n2 : n3));
  for (int64_t i = (int64_t)bid.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gdim.x * blockDim.x)
    m[i] = 0u;
}

// C_B: cells all six of whose faces carry forcing nodes (checked from the
// u list: the west face u(i,j,k) of cell (i,j,k)).
struct CellsK {
  GridView g;
  const int64_t* idx_u;
  const int64_t* count;
  int64_t cap;
  const uint32_t* mu;
  const uint32_t* mv;
  const uint32_t* mw;
  uint32_t* cb_mask;
};
template <bool G = false>
__global__ void k_cells(GArg<CellsK, G> grp_arg_) {
  uint3 bid, gdim;
  const CellsK& P_ = grp_enter<CellsK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  GridView g = P_.g;
  const int64_t* __restrict__ idx_u = P_.idx_u;
  const int64_t* __restrict__ count = P_.count;
  int64_t cap = P_.cap;
  const uint32_t* __restrict__ mu = P_.mu;
  const uint32_t* __restrict__ mv = P_.mv;
  const uint32_t* __restrict__ mw = P_.mw;
  uint32_t* __restrict__ cb_mask = P_.cb_mask;
  int64_t n = count[0];
  if (n > cap) n = cap;
  const int64_t plane = (int64_t)g.nz * g.nx;
  for (int64_t f = (int64_t)bid.x * blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gdim.x * blockDim.x) {
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

// compact nl lists (the three forcing lists, or C_B alone): count, scan and
// emit, one launch each
static void compact(Prof* pf, hipStream_t s, CompactSet S, int nl) {
  int64_t nbmax = 1;
  for (int l = 0; l < nl; ++l) {
    S.nb[l] = (S.nwords[l] + CWB - 1) / CWB;
    if (S.nb[l] > nbmax) nbmax = S.nb[l];
  }
  const dim3 grid((unsigned)nbmax, (unsigned)nl);
  IBM_LAUNCH_G(pf, "tag_count", s, (&k_count<true>), grid, dim3(CT), 0, S,
               k_count<<<grid, CT, 0, s>>>(S));
  IBM_LAUNCH_G(pf, "tag_scan", s, (&k_scan<true>), dim3(nl), dim3(1024), 0, S,
               k_scan<<<nl, 1024, 0, s>>>(S));
  IBM_LAUNCH_G(pf, "tag_emit", s, (&k_emit<true>), grid, dim3(CT), 0, S,
               k_emit<<<grid, CT, 0, s>>>(S));
}

void launch_tag(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nbody,
                int ntri, TagBuffers& tb, uint32_t* flags, double dt) {
  {
    int64_t nmax = tb.nwords_cb;
    for (int c = 0; c < 3; ++c) nmax = tb.nwords[c] > nmax ? tb.nwords[c] : nmax;
    int64_t blocks = (nmax + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    const ZeroMasksK Z{tb.mask[0], tb.nwords[0], tb.mask[1], tb.nwords[1],
                       tb.mask[2], tb.nwords[2], tb.cb_mask, tb.nwords_cb};
    const dim3 zg((unsigned)blocks, 4);
    IBM_LAUNCH_G(pf, "fill_u32", s, (&k_zero_masks<true>), zg, dim3(256), 0, Z,
                 k_zero_masks<<<zg, 256, 0, s>>>(Z));
  }
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
    a.dt = dt;
    dim3 grid((ntri + TAG_TPB - 1) / TAG_TPB, 3);
    a.pass = 0;
    IBM_LAUNCH_G(pf, "tag_pairs", s, (&k_tag_pairs<true>), grid, dim3(64 * TAG_TPB), 0, a,
                 k_tag_pairs<<<grid, 64 * TAG_TPB, 0, s>>>(a));
    a.pass = 1;
    IBM_LAUNCH_G(pf, "tag_pairs", s, (&k_tag_pairs<true>), grid, dim3(64 * TAG_TPB), 0, a,
                 k_tag_pairs<<<grid, 64 * TAG_TPB, 0, s>>>(a));
  }
  // the three forcing lists in one pass; each list has its own block sums
  // (tb.bsum_stride values apart)
  CompactSet S{};
  S.cap = tb.cap;
  S.flags = flags;
  for (int c = 0; c < 3; ++c) {
    S.mask[c] = tb.mask[c];
    S.nwords[c] = tb.nwords[c];
    S.bsum[c] = tb.block_sums + c * tb.bsum_stride;
    S.idx[c] = tb.idx[c];
    S.tri[c] = tb.tri[c];
    S.best_d[c] = tb.best_d[c];
    S.best_t[c] = tb.best_t[c];
    S.count[c] = tb.count + c;
  }
  compact(pf, s, S, 3);
  const CellsK CK{g, tb.idx[0], tb.count, tb.cap, tb.mask[0], tb.mask[1], tb.mask[2], tb.cb_mask};
  IBM_LAUNCH_G(pf, "tag_cells", s, (&k_cells<true>), dim3(1024), dim3(256), 0, CK,
               k_cells<<<1024, 256, 0, s>>>(CK));
  CompactSet B{};
  B.cap = tb.cap;
  B.flags = flags;
  B.mask[0] = tb.cb_mask;
  B.nwords[0] = tb.nwords_cb;
  B.bsum[0] = tb.block_sums;
  B.idx[0] = tb.cb;
  B.count[0] = tb.count + 3;
  compact(pf, s, B, 1);
}

}  // namespace ibm
