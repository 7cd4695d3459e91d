// Two-sided Eulerian IB forcing (paper Eqs. IB_step, probe and new_IB).
//
// One thread per forcing node of the sorted list: recompute the wall point X
// on the forcing triangle and N = x - X; cast the probe x^e = X + h N/|N| with
// h twice the local cell diagonal; interpolate the same velocity component at
// x^e trilinearly on its own lattice (walls act as nodes); blend
// u^f = (1 - a) U + a u^e with a = |N|/h and U the barycentric wall velocity.
// A node on the surface (|N| = 0) takes U.  All values are computed from the
// unmodified field into a buffer and scattered by a second kernel (Jacobi), so
// the result does not depend on the scheduling of the threads.
#pragma clang fp contract(off)

#include "geom.h"

namespace ibm {

struct ForceK {
  GridView g;
  const BodyDev* bodies;
  int nbody;
  const int64_t* idx[3];
  const int32_t* tri[3];
  const int64_t* count;
  int64_t cap;
  double* field[3];
  double* vals;  // 3 * cap
  uint32_t* flags;
};

// ceil(a / b) for b > 0
__device__ __forceinline__ int ceil_div(int a, int b) {
  return a >= 0 ? (a + b - 1) / b : -((-a) / b);
}

__device__ double trilinear(const GridView& g, const Lattice& L, int c, const double* f,
                            const double xe[3], int64_t self, bool* bad) {
  const double sx = xe[0] / g.dx - L.ox;
  const double fx = floor(sx);
  const double tx = sx - fx;
  const double sz = xe[2] / g.dz - L.oz;
  const double fz = floor(sz);
  const double tz = sz - fz;
  const int ix = (int)fx, iz = (int)fz;
  int ey = upper_bound(L.ext, L.next, xe[1]) - 1;
  if (ey < 0) ey = 0;
  if (ey > L.next - 2) ey = L.next - 2;
  const double ty = (xe[1] - L.ext[ey]) / (L.ext[ey + 1] - L.ext[ey]);
  const int64_t plane = (int64_t)g.nz * g.nx;
  double out = 0.0;
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? tx : 1.0 - tx;
    const int ii = wrapi(ix + a, g.nx);
    for (int b = 0; b < 2; ++b) {
      const double wy = b ? ty : 1.0 - ty;
      const int ee = ey + b;
      const int j = (c == 1) ? ee : ee - 1;
      const bool wall = (c == 1) ? false : (ee == 0 || ee == g.ny + 1);
      for (int d = 0; d < 2; ++d) {
        const double wz = d ? tz : 1.0 - tz;
        const int kk = wrapi(iz + d, g.nz);
        const int64_t n = (int64_t)j * plane + (int64_t)kk * g.nx + ii;
        const double val = wall ? 0.0 : f[n];
        out += (wx * wy * wz) * val;
        if (!wall && n == self) *bad = true;
      }
    }
  }
  return out;
}

template <bool G = false>
__global__ __launch_bounds__(256) void k_force_compute(GArg<ForceK, G> grp_arg_) {
  uint3 bid, gdim;
  const ForceK& a = grp_enter<ForceK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  const int c = bid.y;
  int64_t n = a.count[c];
  if (n > a.cap) n = a.cap;
  const GridView& g = a.g;
  const Lattice L = lattice(g, c);
  const int64_t plane = (int64_t)g.nz * g.nx;
  for (int64_t f = (int64_t)bid.x * blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gdim.x * blockDim.x) {
    const int64_t node = a.idx[c][f];
    const int t = a.tri[c][f];
    double A[3], B[3], C[3];
    const double* vel;
    int vid[3];
    load_triangle(a.bodies, a.nbody, t, A, B, C, &vel, vid);
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(A[d], fmin(B[d], C[d]));
      hi[d] = fmax(A[d], fmax(B[d], C[d]));
    }
    const Box bx = candidate_box(g, L, lo, hi);
    const int i = (int)(node % g.nx);
    const int k = (int)((node / g.nx) % g.nz);
    const int j = (int)(node / plane);
    // the periodic image of the node used by the tagging of this triangle
    const int iu = i + g.nx * ceil_div(bx.i0 - i, g.nx);
    const int ku = k + g.nz * ceil_div(bx.k0 - k, g.nz);
    const int e = (c == 1) ? j : j + 1;
    const double p[3] = {((double)iu + L.ox) * g.dx, L.ext[e], ((double)ku + L.oz) * g.dz};
    const ClosestPt X = closest_point(p, A, B, C);
    const double N0 = p[0] - X.x[0], N1 = p[1] - X.x[1], N2 = p[2] - X.x[2];
    const double n2 = dot3(N0, N1, N2, N0, N1, N2);
    const double U = (X.w[0] * vel[3 * vid[0] + c] + X.w[1] * vel[3 * vid[1] + c]) +
                     X.w[2] * vel[3 * vid[2] + c];
    double val = U;
    if (n2 != 0.0) {
      const double nn = sqrt(n2);
      const double dyl = (c == 1) ? g.dyc[j] : g.dy[j];
      const double h = 2.0 * sqrt(g.dx * g.dx + g.dz * g.dz + dyl * dyl);
      const double xe[3] = {X.x[0] + h * (N0 / nn), X.x[1] + h * (N1 / nn),
                            X.x[2] + h * (N2 / nn)};
      const double w = nn / h;
      bool bad = false;
      if (xe[1] < L.ext[0] || xe[1] > L.ext[L.next - 1]) {
        bad = true;
      } else {
        const double ue = trilinear(g, L, c, a.field[c], xe, node, &bad);
        val = (1.0 - w) * U + w * ue;
      }
      if (bad) atomicOr(a.flags, FLAG_GEOM);
    }
    a.vals[c * a.cap + f] = val;
  }
}

template <bool G = false>
__global__ __launch_bounds__(256) void k_force_scatter(GArg<ForceK, G> grp_arg_) {
  uint3 bid, gdim;
  const ForceK& a = grp_enter<ForceK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  const int c = bid.y;
  int64_t n = a.count[c];
  if (n > a.cap) n = a.cap;
  for (int64_t f = (int64_t)bid.x * blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gdim.x * blockDim.x)
    a.field[c][a.idx[c][f]] = a.vals[c * a.cap + f];
}

// No-slip (transpiration) error at every forcing node (paper Sec. 4.4: the
// flow velocity interpolated on the surface with the forcing interpolator of
// Eq. new_IB, against the wall velocity): with the wall point X, N, the probe
// x^e and a = |N|/h exactly as in the forcing, the flow extrapolated to the
// wall is (u(x^f) - a u(x^e)) / (1 - a) (u(x^f) itself when |N| = 0); the
// node's error |that - U| goes to vals[c cap + f].
__global__ __launch_bounds__(256) void k_noslip(ForceK a) {
  const int c = blockIdx.y;
  int64_t n = a.count[c];
  if (n > a.cap) n = a.cap;
  const GridView& g = a.g;
  const Lattice L = lattice(g, c);
  const int64_t plane = (int64_t)g.nz * g.nx;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = a.idx[c][f];
    const int t = a.tri[c][f];
    double A[3], B[3], C[3];
    const double* vel;
    int vid[3];
    load_triangle(a.bodies, a.nbody, t, A, B, C, &vel, vid);
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(A[d], fmin(B[d], C[d]));
      hi[d] = fmax(A[d], fmax(B[d], C[d]));
    }
    const Box bx = candidate_box(g, L, lo, hi);
    const int i = (int)(node % g.nx);
    const int k = (int)((node / g.nx) % g.nz);
    const int j = (int)(node / plane);
    const int iu = i + g.nx * ceil_div(bx.i0 - i, g.nx);
    const int ku = k + g.nz * ceil_div(bx.k0 - k, g.nz);
    const int e = (c == 1) ? j : j + 1;
    const double p[3] = {((double)iu + L.ox) * g.dx, L.ext[e], ((double)ku + L.oz) * g.dz};
    const ClosestPt X = closest_point(p, A, B, C);
    const double N0 = p[0] - X.x[0], N1 = p[1] - X.x[1], N2 = p[2] - X.x[2];
    const double n2 = dot3(N0, N1, N2, N0, N1, N2);
    const double U = (X.w[0] * vel[3 * vid[0] + c] + X.w[1] * vel[3 * vid[1] + c]) +
                     X.w[2] * vel[3 * vid[2] + c];
    const double uf = a.field[c][node];
    double wall = uf;
    if (n2 != 0.0) {
      const double nn = sqrt(n2);
      const double dyl = (c == 1) ? g.dyc[j] : g.dy[j];
      const double h = 2.0 * sqrt(g.dx * g.dx + g.dz * g.dz + dyl * dyl);
      const double xe[3] = {X.x[0] + h * (N0 / nn), X.x[1] + h * (N1 / nn),
                            X.x[2] + h * (N2 / nn)};
      const double w = nn / h;
      bool bad = false;
      if (xe[1] < L.ext[0] || xe[1] > L.ext[L.next - 1]) {
        bad = true;
      } else {
        const double ue = trilinear(g, L, c, a.field[c], xe, node, &bad);
        wall = (uf - w * ue) / (1.0 - w);
      }
      if (bad) atomicOr(a.flags, FLAG_GEOM);
    }
    a.vals[c * a.cap + f] = fabs(wall - U);
  }
}

// per component: the mean of vals[c cap + f] over its forcing nodes (0
// without any), summed in a fixed order (one block per component)
__global__ __launch_bounds__(256) void k_noslip_mean(const double* __restrict__ vals,
                                                      const int64_t* __restrict__ count,
                                                      int64_t cap, double* __restrict__ out) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  int64_t n = count[c];
  if (n > cap) n = cap;
  double acc = 0.0;
  for (int64_t f = threadIdx.x; f < n; f += 256) acc += vals[c * cap + f];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = (n > 0) ? sh[0] / (double)n : 0.0;
}

// Pressure on the boundary cells (paper Sec. 2, after Eq. q_F: rebuilt from
// the surrounding field with the strategy of the forcing, as post-processing).
// For a C_B cell: the wall point X is the closest point of the cell centre on
// the forcing triangles of the cell's six faces (least |N|^2, ties to the
// lowest triangle id; the centre's periodic image nearest the triangle's
// centroid); the probe x^e = X + h N/|N|, h twice the cell's diagonal; the
// wall has no pressure value, so the cell takes p(x^e) (zero normal
// gradient), trilinear on the cell-centre lattice, constant beyond the first
// and last centres.  A centre on the surface takes the mean of the probes on
// both sides along the triangle's normal.
template <typename T>
struct PcbK {
  GridView g;
  const BodyDev* bodies;
  int nbody;
  const int64_t* idx[3];
  const int32_t* tri[3];
  const int64_t* cb;
  const int64_t* count;
  int64_t cap;
  const T* p;
  double* out;
  int64_t out_cap;
  uint32_t* flags;
};

// position of node in the sorted list idx[0..n), or -1
__device__ __forceinline__ int64_t find_node(const int64_t* idx, int64_t n, int64_t node) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (idx[mid] < node) lo = mid + 1; else hi = mid;
  }
  return (lo < n && idx[lo] == node) ? lo : -1;
}

template <typename T>
__device__ double p_trilinear(const GridView& g, const T* p, double x, double y, double z) {
  const double sx = x / g.dx - 0.5;
  const double fx = floor(sx);
  const double tx = sx - fx;
  const double sz = z / g.dz - 0.5;
  const double fz = floor(sz);
  const double tz = sz - fz;
  const int ix = (int)fx, iz = (int)fz;
  int ey = upper_bound(g.yc, g.ny, y) - 1;
  if (ey < 0) ey = 0;
  if (ey > g.ny - 2) ey = g.ny - 2;
  double ty = (y - g.yc[ey]) / (g.yc[ey + 1] - g.yc[ey]);
  ty = ty < 0.0 ? 0.0 : (ty > 1.0 ? 1.0 : ty);
  const int64_t plane = (int64_t)g.nz * g.nx;
  double out = 0.0;
  for (int a = 0; a < 2; ++a) {
    const double wx = a ? tx : 1.0 - tx;
    const int ii = wrapi(ix + a, g.nx);
    for (int b = 0; b < 2; ++b) {
      const double wy = b ? ty : 1.0 - ty;
      for (int d = 0; d < 2; ++d) {
        const double wz = d ? tz : 1.0 - tz;
        const int kk = wrapi(iz + d, g.nz);
        out += (wx * wy * wz) * (double)p[(int64_t)(ey + b) * plane + (int64_t)kk * g.nx + ii];
      }
    }
  }
  return out;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pressure_cb(PcbK<T> a) {
  const GridView& g = a.g;
  int64_t n = a.count[3];
  if (n > a.cap) n = a.cap;
  if (n > a.out_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(a.flags, FLAG_CAPACITY);
    n = a.out_cap;
  }
  const int64_t plane = (int64_t)g.nz * g.nx;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cell = a.cb[f];
    const int i = (int)(cell % g.nx);
    const int k = (int)((cell / g.nx) % g.nz);
    const int j = (int)(cell / plane);
    const int64_t node[6] = {cell, (int64_t)j * plane + (int64_t)k * g.nx + wrapi(i + 1, g.nx),
                             cell, cell + plane,
                             cell, (int64_t)j * plane + (int64_t)wrapi(k + 1, g.nz) * g.nx + i};
    const double ctr[3] = {((double)i + 0.5) * g.dx, g.yc[j], ((double)k + 0.5) * g.dz};
    double bn2 = 0.0, bX[3] = {0.0, 0.0, 0.0}, bp[3] = {0.0, 0.0, 0.0};
    double bA[3] = {0, 0, 0}, bB[3] = {0, 0, 0}, bC[3] = {0, 0, 0};
    int bt = -1;
    for (int q = 0; q < 6; ++q) {
      const int c = q >> 1;
      int64_t nc = a.count[c];
      if (nc > a.cap) nc = a.cap;
      const int64_t pos = find_node(a.idx[c], nc, node[q]);
      if (pos < 0) {  // a C_B face must be a forcing node
        atomicOr(a.flags, FLAG_GEOM);
        continue;
      }
      const int t = a.tri[c][pos];
      double A[3], B[3], C[3];
      const double* vel;
      int vid[3];
      load_triangle(a.bodies, a.nbody, t, A, B, C, &vel, vid);
      const double cx = (A[0] + B[0] + C[0]) / 3.0, cz = (A[2] + B[2] + C[2]) / 3.0;
      const double pc[3] = {ctr[0] + g.lx * rint((cx - ctr[0]) / g.lx), ctr[1],
                            ctr[2] + g.lz * rint((cz - ctr[2]) / g.lz)};
      const ClosestPt X = closest_point(pc, A, B, C);
      const double N0 = pc[0] - X.x[0], N1 = pc[1] - X.x[1], N2 = pc[2] - X.x[2];
      const double n2 = dot3(N0, N1, N2, N0, N1, N2);
      if (bt < 0 || n2 < bn2 || (n2 == bn2 && t < bt)) {
        bt = t;
        bn2 = n2;
        for (int d = 0; d < 3; ++d) {
          bX[d] = X.x[d];
          bp[d] = pc[d];
          bA[d] = A[d];
          bB[d] = B[d];
          bC[d] = C[d];
        }
      }
    }
    if (bt < 0) continue;
    const double h = 2.0 * sqrt(g.dx * g.dx + g.dz * g.dz + g.dy[j] * g.dy[j]);
    double val;
    if (bn2 != 0.0) {
      const double nn = sqrt(bn2);
      val = p_trilinear(g, a.p, bX[0] + h * ((bp[0] - bX[0]) / nn),
                        bX[1] + h * ((bp[1] - bX[1]) / nn), bX[2] + h * ((bp[2] - bX[2]) / nn));
    } else {
      const double e1[3] = {bB[0] - bA[0], bB[1] - bA[1], bB[2] - bA[2]};
      const double e2[3] = {bC[0] - bA[0], bC[1] - bA[1], bC[2] - bA[2]};
      double nr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                      e1[0] * e2[1] - e1[1] * e2[0]};
      const double len = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
      for (int d = 0; d < 3; ++d) nr[d] /= len;
      const double plus = p_trilinear(g, a.p, bX[0] + h * nr[0], bX[1] + h * nr[1], bX[2] + h * nr[2]);
      const double minus = p_trilinear(g, a.p, bX[0] - h * nr[0], bX[1] - h * nr[1], bX[2] - h * nr[2]);
      val = 0.5 * (plus + minus);
    }
    a.out[f] = val;
  }
}

void launch_pressure_cb(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies,
                        int nbody, const TagBuffers& tb, const void* p, int fp32, double* out,
                        int64_t out_cap, uint32_t* flags) {
  int blocks = (int)((tb.cap + 255) / 256);
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  auto fill = [&](auto K) {
    K.g = g;
    K.bodies = bodies;
    K.nbody = nbody;
    for (int c = 0; c < 3; ++c) {
      K.idx[c] = tb.idx[c];
      K.tri[c] = tb.tri[c];
    }
    K.cb = tb.cb;
    K.count = tb.count;
    K.cap = tb.cap;
    K.out = out;
    K.out_cap = out_cap;
    K.flags = flags;
    return K;
  };
  if (fp32) {
    PcbK<float> K = fill(PcbK<float>{});
    K.p = static_cast<const float*>(p);
    IBM_LAUNCH(pf, "pressure_cb", s, k_pressure_cb<float><<<blocks, 256, 0, s>>>(K));
  } else {
    PcbK<double> K = fill(PcbK<double>{});
    K.p = static_cast<const double*>(p);
    IBM_LAUNCH(pf, "pressure_cb", s, k_pressure_cb<double><<<blocks, 256, 0, s>>>(K));
  }
}

void launch_noslip(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nbody,
                   const TagBuffers& tb, const double* const* fields, double* vals, double* out,
                   uint32_t* flags) {
  ForceK a;
  a.g = g;
  a.bodies = bodies;
  a.nbody = nbody;
  for (int c = 0; c < 3; ++c) {
    a.idx[c] = tb.idx[c];
    a.tri[c] = tb.tri[c];
    a.field[c] = const_cast<double*>(fields[c]);
  }
  a.count = tb.count;
  a.cap = tb.cap;
  a.vals = vals;
  a.flags = flags;
  int blocks = (int)((tb.cap + 255) / 256);
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  IBM_LAUNCH(pf, "noslip", s, k_noslip<<<dim3(blocks, 3), 256, 0, s>>>(a));
  IBM_LAUNCH(pf, "noslip_mean", s, k_noslip_mean<<<3, 256, 0, s>>>(vals, tb.count, tb.cap, out));
}

void launch_force(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nbody,
                  const TagBuffers& tb, double* const* fields, double* vals, uint32_t* flags) {
  ForceK a;
  a.g = g;
  a.bodies = bodies;
  a.nbody = nbody;
  for (int c = 0; c < 3; ++c) {
    a.idx[c] = tb.idx[c];
    a.tri[c] = tb.tri[c];
    a.field[c] = fields[c];
  }
  a.count = tb.count;
  a.cap = tb.cap;
  a.vals = vals;
  a.flags = flags;
  int blocks = (int)((tb.cap + 255) / 256);
  if (blocks > 512) blocks = 512;
  if (blocks < 1) blocks = 1;
  dim3 grid(blocks, 3);
  IBM_LAUNCH_G(pf, "force_compute", s, (&k_force_compute<true>), grid, dim3(256), 0, a,
               k_force_compute<<<grid, 256, 0, s>>>(a));
  IBM_LAUNCH_G(pf, "force_scatter", s, (&k_force_scatter<true>), grid, dim3(256), 0, a,
               k_force_scatter<<<grid, 256, 0, s>>>(a));
}

}  // namespace ibm
