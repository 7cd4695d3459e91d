// Approximate-factorisation line solves of the predictor (paper Sec. 2:
// "approximate factorization of L, yielding three tridiagonal systems per
// direction"):
//   (I - beta L_x) w1 = R   cyclic in x, constant coefficients
//   (I - beta L_z) w2 = w1  cyclic in z, constant coefficients
//   (I - beta L_y) du = w2  Dirichlet walls, stretched spacing
// with identity rows on the forcing nodes (the stencil never crosses the
// interface, Sec. 3.1 and Fig. 3), then u <- u + du.
//
// One lane per line; consecutive lanes take consecutive lines so that the
// z- and y-sweeps read contiguous row segments (coalesced over x).  Lines
// without forcing nodes (all but a few) use the factorisation of the
// mask-free matrix, which is the same for every line and is read from small
// tables through the scalar cache; for the cyclic directions the
// Sherman-Morrison correction is folded into the two sweeps (the weights W
// give y_0 = sum_i W_i d'_i during the forward sweep).  Lines that hold
// forcing nodes are solved in general form: a cyclic line is cut open at its
// first forcing node (whose value is 0) and the Thomas recursion restarts at
// every identity row; its c' coefficients go to a scratch array.
// d' overwrites the right-hand side in place between the two sweeps.
#include "geom.h"

namespace ibm {

constexpr int CH = 8;  // elements per lane per chunk (loads issued together)

// mask-free cyclic line: d[0..n-1] with stride s -> solution in place
__device__ __forceinline__ void cyclic_fast(double* __restrict__ d, int64_t s, int n,
                                            const CyclicTab& t) {
  double prev = 0.0, acc = 0.0;
  for (int i0 = 0; i0 < n; i0 += CH) {
    double buf[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (i0 + q < n) buf[q] = d[(int64_t)(i0 + q) * s];
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (i0 + q < n) {
        const double dp = (buf[q] - t.a * prev) * t.inv[i0 + q];
        acc += t.W[i0 + q] * dp;
        buf[q] = dp;
        prev = dp;
      }
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (i0 + q < n) d[(int64_t)(i0 + q) * s] = buf[q];
  }
  const double fact = (acc + t.ratio * prev) * t.fden_inv;
  double ynext = 0.0;
  for (int i1 = n; i1 > 0; i1 -= CH) {
    double buf[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (i1 - 1 - q >= 0) buf[q] = d[(int64_t)(i1 - 1 - q) * s];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int i = i1 - 1 - q;
      if (i >= 0) {
        const double y = buf[q] - t.cp[i] * ynext;
        buf[q] = y - fact * t.Z[i];
        ynext = y;
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (i1 - 1 - q >= 0) d[(int64_t)(i1 - 1 - q) * s] = buf[q];
  }
}

// cyclic line with identity rows; node(i) = node0 + i*s for the mask
__device__ void cyclic_general(double* __restrict__ d, double* __restrict__ cps, int64_t s,
                               int n, const CyclicTab& t, const uint32_t* __restrict__ mask,
                               int64_t node0) {
  int f0 = 0;
  for (int i = 0; i < n; ++i)
    if (test_bit(mask, node0 + (int64_t)i * s)) {
      f0 = i;
      break;
    }
  double cpp = 0.0, dpp = 0.0;
  for (int q = 1; q < n; ++q) {
    int i = f0 + q;
    if (i >= n) i -= n;
    const int64_t o = (int64_t)i * s;
    double cp, dp;
    if (test_bit(mask, node0 + o)) {
      cp = 0.0;
      dp = 0.0;
    } else {
      const double m = t.b - t.a * cpp;
      cp = t.c / m;
      dp = (d[o] - t.a * dpp) / m;
    }
    cps[o] = cp;
    d[o] = dp;
    cpp = cp;
    dpp = dp;
  }
  double xn = 0.0;
  for (int q = n - 1; q >= 1; --q) {
    int i = f0 + q;
    if (i >= n) i -= n;
    const int64_t o = (int64_t)i * s;
    const double x = d[o] - cps[o] * xn;
    d[o] = x;
    xn = x;
  }
  d[(int64_t)f0 * s] = 0.0;
}

struct AdiK {
  GridView g;
  double* d;
  double* u;  // y-sweep: field updated with du
  const uint8_t* flag;
  const uint32_t* mask;
  double* scratch;
  CyclicTab ct;
  YTab yt;
  int j0, nj;  // first node plane and number of planes (x, z sweeps)
};

__global__ __launch_bounds__(256) void k_adi_x(AdiK K) {
  const GridView& g = K.g;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= (int64_t)K.nj * g.nz) return;
  const int j = K.j0 + (int)(line / g.nz);
  const int k = (int)(line % g.nz);
  const int64_t base = ((int64_t)j * g.nz + k) * g.nx;
  if (!K.flag[(int64_t)j * g.nz + k])
    cyclic_fast(K.d + base, 1, g.nx, K.ct);
  else
    cyclic_general(K.d + base, K.scratch + base, 1, g.nx, K.ct, K.mask, base);
}

__global__ __launch_bounds__(256) void k_adi_z(AdiK K) {
  const GridView& g = K.g;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= (int64_t)K.nj * g.nx) return;
  const int j = K.j0 + (int)(line / g.nx);
  const int i = (int)(line % g.nx);
  const int64_t base = (int64_t)j * g.nz * g.nx + i;
  if (!K.flag[(int64_t)j * g.nx + i])
    cyclic_fast(K.d + base, g.nx, g.nz, K.ct);
  else
    cyclic_general(K.d + base, K.scratch + base, g.nx, g.nz, K.ct, K.mask, base);
}

__global__ __launch_bounds__(256) void k_adi_y(AdiK K) {
  const GridView& g = K.g;
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= (int64_t)g.nz * g.nx) return;
  const int64_t plane = (int64_t)g.nz * g.nx;
  const YTab& t = K.yt;
  const int n = t.n;
  const int64_t base = (int64_t)t.j0 * plane + line;  // node of row 0
  double* __restrict__ d = K.d + base;
  double* __restrict__ u = K.u + base;
  if (!K.flag[line]) {
    double prev = 0.0;
    for (int r0 = 0; r0 < n; r0 += CH) {
      double buf[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (r0 + q < n) buf[q] = d[(int64_t)(r0 + q) * plane];
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (r0 + q < n) {
          const double dp = (buf[q] - t.a[r0 + q] * prev) * t.inv[r0 + q];
          buf[q] = dp;
          prev = dp;
        }
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (r0 + q < n) d[(int64_t)(r0 + q) * plane] = buf[q];
    }
    double xn = 0.0;
    for (int r1 = n; r1 > 0; r1 -= CH) {
      double buf[CH], ub[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (r1 - 1 - q >= 0) {
          buf[q] = d[(int64_t)(r1 - 1 - q) * plane];
          ub[q] = u[(int64_t)(r1 - 1 - q) * plane];
        }
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int r = r1 - 1 - q;
        if (r >= 0) {
          const double x = buf[q] - t.cp[r] * xn;
          ub[q] += x;
          xn = x;
        }
      }
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (r1 - 1 - q >= 0) u[(int64_t)(r1 - 1 - q) * plane] = ub[q];
    }
  } else {
    double* __restrict__ cps = K.scratch + base;
    double cpp = 0.0, dpp = 0.0;
    for (int r = 0; r < n; ++r) {
      const int64_t o = (int64_t)r * plane;
      double cp, dp;
      if (test_bit(K.mask, base + o)) {
        cp = 0.0;
        dp = 0.0;
      } else {
        const double m = t.b[r] - t.a[r] * cpp;
        cp = t.c[r] / m;
        dp = (d[o] - t.a[r] * dpp) / m;
      }
      cps[o] = cp;
      d[o] = dp;
      cpp = cp;
      dpp = dp;
    }
    double xn = 0.0;
    for (int r = n - 1; r >= 0; --r) {
      const int64_t o = (int64_t)r * plane;
      const double x = d[o] - cps[o] * xn;
      u[o] += x;
      xn = x;
    }
  }
}

void launch_adi_x(Prof* pf, hipStream_t s, const GridView& g, int comp, double* d,
                  const uint8_t* xflag, const uint32_t* mask, const CyclicTab& t,
                  double* scratch) {
  AdiK K{};
  K.g = g;
  K.d = d;
  K.flag = xflag;
  K.mask = mask;
  K.scratch = scratch;
  K.ct = t;
  K.j0 = (comp == 1) ? 1 : 0;
  K.nj = (comp == 1) ? g.ny - 1 : g.ny;
  const int64_t nl = (int64_t)K.nj * g.nz;
  IBM_LAUNCH(pf, "adi_x", s, k_adi_x<<<(int)((nl + 255) / 256), 256, 0, s>>>(K));
}

void launch_adi_z(Prof* pf, hipStream_t s, const GridView& g, int comp, double* d,
                  const uint8_t* zflag, const uint32_t* mask, const CyclicTab& t,
                  double* scratch) {
  AdiK K{};
  K.g = g;
  K.d = d;
  K.flag = zflag;
  K.mask = mask;
  K.scratch = scratch;
  K.ct = t;
  K.j0 = (comp == 1) ? 1 : 0;
  K.nj = (comp == 1) ? g.ny - 1 : g.ny;
  const int64_t nl = (int64_t)K.nj * g.nx;
  IBM_LAUNCH(pf, "adi_z", s, k_adi_z<<<(int)((nl + 255) / 256), 256, 0, s>>>(K));
}

void launch_adi_y(Prof* pf, hipStream_t s, const GridView& g, int comp, const double* d,
                  double* u, const uint8_t* yflag, const uint32_t* mask, const YTab& t,
                  double* scratch) {
  AdiK K{};
  K.g = g;
  K.d = const_cast<double*>(d);
  K.u = u;
  K.flag = yflag;
  K.mask = mask;
  K.scratch = scratch;
  K.yt = t;
  (void)comp;
  const int64_t nl = (int64_t)g.nz * g.nx;
  IBM_LAUNCH(pf, "adi_y", s, k_adi_y<<<(int)((nl + 255) / 256), 256, 0, s>>>(K));
}

}  // namespace ibm
