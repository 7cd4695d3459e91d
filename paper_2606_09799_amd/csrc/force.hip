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

__global__ __launch_bounds__(256) void k_force_compute(ForceK a) {
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

__global__ __launch_bounds__(256) void k_force_scatter(ForceK a) {
  const int c = blockIdx.y;
  int64_t n = a.count[c];
  if (n > a.cap) n = a.cap;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gridDim.x * blockDim.x)
    a.field[c][a.idx[c][f]] = a.vals[c * a.cap + f];
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
  IBM_LAUNCH(pf, "force_compute", s, k_force_compute<<<grid, 256, 0, s>>>(a));
  IBM_LAUNCH(pf, "force_scatter", s, k_force_scatter<<<grid, 256, 0, s>>>(a));
}

}  // namespace ibm
