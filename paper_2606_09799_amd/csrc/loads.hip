// Hydrodynamic loads on the bodies of the last tagging (paper Sec. 3.3).
//
// One thread per triangle (marker): the centroid X, unit normal n (the
// triangle's winding) and area A; the probe point x_e = X + s h n (side
// s = +1, and also -1 for a two-sided body), h twice the diagonal of the
// grid cell that holds X; for p and each velocity component a weighted
// least-squares fit of a quadratic around x_e on that quantity's own
// lattice (the 4 x 4 x 4 nodes around x_e, wall points included for the
// velocity, only nodes in front of the marker's tangent plane, only fluid
// cells for p; weights exp(-|d|^2), d = (x - x_e)/D, D the largest spacing
// of the cell), solved by Cholesky on the 10 x 10 normal equations (their
// condition number is about 10 with this scaling); then
//   p_X = p - h dp/dn + h^2/2 d2p/dn2,   G_X = G - h dG/dn
// at x_e, and the traction t = -p_X n_s + (G_X + G_X^T) n_s / Re, summed over
// the sides.  A second kernel sums t A and (X - pole) x t A per body, in a
// fixed order (one block per body).
//
// The marker geometry, the probe point and the stencil decisions (the floor
// that places the 4 x 4 x 4 window, the y bracket, the tangent-plane test)
// use IEEE binary64 +, -, *, / in the written order, without contraction
// into FMA, so that a probe point lying exactly on a lattice line takes the
// same window as a plain evaluation of the same expressions.
#include "lanes.h"

#pragma clang fp contract(off)

namespace ibm {

struct LoadsK {
  GridView g;
  const BodyDev* bodies;
  int nb, ntri;
  const double* u;
  const double* v;
  const double* w;
  const void* p;
  int p32;
  const uint32_t* cb_mask;  // C_B cells of the last tagging (NULL: none)
  const int32_t* sides;     // nb: 1 (closed body) or 2 (two-sided)
  double inv_re;
  double* traction;         // 3 ntri
};

// packed lower triangle of the 10 x 10 normal matrix: (a, b), a >= b
__device__ __forceinline__ constexpr int tri_ix(int a, int b) { return a * (a + 1) / 2 + b; }

// One fit: value, gradient and Hessian at xe of quantity q (0-2: velocity
// components, 3: pressure).
struct Fit {
  double val, gr[3], H[3][3];
};

__device__ __forceinline__ double p_at(const LoadsK& K, int64_t c) {
  return K.p32 ? (double)static_cast<const float*>(K.p)[c] : static_cast<const double*>(K.p)[c];
}

__device__ Fit mls_fit(const LoadsK& K, int q, const double xe[3], const double X[3],
                       const double ns[3], double D) {
  const GridView& g = K.g;
  // lattice: offsets in x and z, y heights (nodes of the stencil window)
  const double ox = (q == 0) ? 0.0 : 0.5, oz = (q == 2) ? 0.0 : 0.5;
  int nyl;  // lattice heights: p: ny centres; v: ny+1 faces; u, w: ny+2 (walls + centres)
  const double* ys;
  if (q == 3) {
    ys = g.yc;
    nyl = g.ny;
  } else if (q == 1) {
    ys = g.yf;
    nyl = g.ny + 1;
  } else {
    ys = g.extuw;
    nyl = g.ny + 2;
  }
  // bracket: the largest lattice index e with ys[e] <= xe_y
  int lo = 0, hi = nyl;  // ys[lo] <= y < ys[hi] once narrowed
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ys[mid] <= xe[1]) lo = mid; else hi = mid;
  }
  int e0 = (xe[1] < ys[0]) ? -2 : lo - 1;
  if (e0 < 0) e0 = 0;
  if (e0 > nyl - 4) e0 = nyl - 4;
  const int i0 = (int)floor(xe[0] / g.dx - ox) - 1;
  const int k0 = (int)floor(xe[2] / g.dz - oz) - 1;
  const double iD = 1.0 / D;
  double A[55], b[10];
#pragma unroll
  for (int a = 0; a < 55; ++a) A[a] = 0.0;
#pragma unroll
  for (int a = 0; a < 10; ++a) b[a] = 0.0;
  const int64_t plane = (int64_t)g.nz * g.nx;
  for (int e = e0; e < e0 + 4; ++e) {
    const double py = ys[e];
    // array row of the lattice height (-1: a wall point of u or w, value 0)
    const int jr = (q == 0 || q == 2) ? ((e == 0 || e == g.ny + 1) ? -1 : e - 1) : e;
    for (int kk = k0; kk < k0 + 4; ++kk) {
      const double pz = (kk + oz) * g.dz;
      const int km = ((kk % g.nz) + g.nz) % g.nz;
      for (int ii = i0; ii < i0 + 4; ++ii) {
        const double px = (ii + ox) * g.dx;
        if ((px - X[0]) * ns[0] + (py - X[1]) * ns[1] + (pz - X[2]) * ns[2] <= 0.0) continue;
        const int im = ((ii % g.nx) + g.nx) % g.nx;
        double val = 0.0;
        if (jr >= 0) {
          const int64_t c = (int64_t)jr * plane + (int64_t)km * g.nx + im;
          if (q == 3) {
            if (K.cb_mask && test_bit(K.cb_mask, c)) continue;
            val = p_at(K, c);
          } else {
            val = (q == 0 ? K.u : (q == 1 ? K.v : K.w))[c];
          }
        }
        const double dx = (px - xe[0]) * iD, dy = (py - xe[1]) * iD, dz = (pz - xe[2]) * iD;
        const double wt = exp(-(dx * dx + dy * dy + dz * dz));
        const double P[10] = {1.0, dx, dy, dz, dx * dx, dy * dy, dz * dz, dx * dy, dy * dz, dx * dz};
#pragma unroll
        for (int a = 0; a < 10; ++a) {
          const double wa = wt * P[a];
          b[a] += wa * val;
#pragma unroll
          for (int c2 = 0; c2 <= a; ++c2) A[tri_ix(a, c2)] += wa * P[c2];
        }
      }
    }
  }
  // Cholesky A = L L^T in place, then L y = b, L^T c = y
#pragma unroll
  for (int a = 0; a < 10; ++a) {
#pragma unroll
    for (int c2 = 0; c2 <= a; ++c2) {
      double s = A[tri_ix(a, c2)];
#pragma unroll
      for (int m = 0; m < c2; ++m) s -= A[tri_ix(a, m)] * A[tri_ix(c2, m)];
      A[tri_ix(a, c2)] = (a == c2) ? sqrt(s) : s / A[tri_ix(c2, c2)];
    }
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) {
    double s = b[a];
#pragma unroll
    for (int m = 0; m < a; ++m) s -= A[tri_ix(a, m)] * b[m];
    b[a] = s / A[tri_ix(a, a)];
  }
#pragma unroll
  for (int a = 9; a >= 0; --a) {
    double s = b[a];
#pragma unroll
    for (int m = a + 1; m < 10; ++m) s -= A[tri_ix(m, a)] * b[m];
    b[a] = s / A[tri_ix(a, a)];
  }
  Fit f;
  f.val = b[0];
  f.gr[0] = b[1] * iD;
  f.gr[1] = b[2] * iD;
  f.gr[2] = b[3] * iD;
  const double iD2 = iD * iD;
  f.H[0][0] = 2.0 * b[4] * iD2;
  f.H[1][1] = 2.0 * b[5] * iD2;
  f.H[2][2] = 2.0 * b[6] * iD2;
  f.H[0][1] = f.H[1][0] = b[7] * iD2;
  f.H[1][2] = f.H[2][1] = b[8] * iD2;
  f.H[0][2] = f.H[2][0] = b[9] * iD2;
  return f;
}

__global__ __launch_bounds__(64) void k_loads_markers(LoadsK K) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= K.ntri) return;
  int bi = 0;
  while (bi + 1 < K.nb && m >= K.bodies[bi + 1].toff) ++bi;
  const BodyDev B = K.bodies[bi];
  const int32_t* T = B.tri + 3 * (int64_t)(m - B.toff);
  double P0[3], P1[3], P2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    P0[d] = B.xyz[3 * (int64_t)T[0] + d];
    P1[d] = B.xyz[3 * (int64_t)T[1] + d];
    P2[d] = B.xyz[3 * (int64_t)T[2] + d];
  }
  double X[3], e1[3], e2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    X[d] = (P0[d] + P1[d] + P2[d]) / 3.0;
    e1[d] = P1[d] - P0[d];
    e2[d] = P2[d] - P0[d];
  }
  const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
  const double nrm = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  const double n[3] = {cr[0] / nrm, cr[1] / nrm, cr[2] / nrm};
  const GridView& g = K.g;
  // cell of X in y: the largest j with yf[j] <= y (clamped to 0..ny-1)
  int lo = 0, hi = g.ny + 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (g.yf[mid] <= X[1]) lo = mid; else hi = mid;
  }
  const int j = (lo > g.ny - 1) ? g.ny - 1 : lo;
  const double dyj = g.dy[j];
  const double h = 2.0 * sqrt(g.dx * g.dx + g.dz * g.dz + dyj * dyj);
  const double D = fmax(fmax(g.dx, g.dz), dyj);
  double t[3] = {0.0, 0.0, 0.0};
  const int ns_count = (K.sides[bi] == 2) ? 2 : 1;
  for (int sd = 0; sd < ns_count; ++sd) {
    const double s = sd ? -1.0 : 1.0;
    const double ns[3] = {s * n[0], s * n[1], s * n[2]};
    const double xe[3] = {X[0] + h * ns[0], X[1] + h * ns[1], X[2] + h * ns[2]};
    const Fit fp = mls_fit(K, 3, xe, X, ns, D);
    double Hn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Hn[a] = fp.H[a][0] * ns[0] + fp.H[a][1] * ns[1] + fp.H[a][2] * ns[2];
    const double dpdn = fp.gr[0] * ns[0] + fp.gr[1] * ns[1] + fp.gr[2] * ns[2];
    const double d2pdn2 = Hn[0] * ns[0] + Hn[1] * ns[1] + Hn[2] * ns[2];
    const double pl = fp.val - h * dpdn + 0.5 * h * h * d2pdn2;
    double G[3][3];  // G[i][j] = d u_i / d x_j at X
    for (int c = 0; c < 3; ++c) {
      const Fit fu = mls_fit(K, c, xe, X, ns, D);
#pragma unroll
      for (int a = 0; a < 3; ++a)
        G[c][a] = fu.gr[a] - h * (fu.H[a][0] * ns[0] + fu.H[a][1] * ns[1] + fu.H[a][2] * ns[2]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double sn = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) sn += (G[a][c] + G[c][a]) * ns[c];
      t[a] += -pl * ns[a] + sn * K.inv_re;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) K.traction[3 * (int64_t)m + a] = t[a];
}

// per body: F = sum t A, M = sum (X - pole) x t A, in a fixed order
__global__ __launch_bounds__(256) void k_loads_sum(const BodyDev* bodies, const double* traction,
                                                   const double* pole, double* out) {
  const BodyDev B = bodies[blockIdx.x];
  const double* pl = pole + 3 * blockIdx.x;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int l = threadIdx.x; l < B.nt; l += blockDim.x) {
    const int32_t* T = B.tri + 3 * (int64_t)l;
    double X[3], e1[3], e2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a0 = B.xyz[3 * (int64_t)T[0] + d], a1 = B.xyz[3 * (int64_t)T[1] + d],
                   a2 = B.xyz[3 * (int64_t)T[2] + d];
      X[d] = (a0 + a1 + a2) / 3.0 - pl[d];
      e1[d] = a1 - a0;
      e2[d] = a2 - a0;
    }
    const double cr0 = e1[1] * e2[2] - e1[2] * e2[1], cr1 = e1[2] * e2[0] - e1[0] * e2[2],
                 cr2 = e1[0] * e2[1] - e1[1] * e2[0];
    const double A = 0.5 * sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2);
    const double* t = traction + 3 * (int64_t)(B.toff + l);
    acc[0] += t[0] * A;
    acc[1] += t[1] * A;
    acc[2] += t[2] * A;
    acc[3] += (X[1] * t[2] - X[2] * t[1]) * A;
    acc[4] += (X[2] * t[0] - X[0] * t[2]) * A;
    acc[5] += (X[0] * t[1] - X[1] * t[0]) * A;
  }
  __shared__ double red[6][256];
#pragma unroll
  for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 6) out[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

void launch_loads(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nb,
                  int ntri, const double* u, const double* v, const double* w, const void* p,
                  int p32, const uint32_t* cb_mask, const int32_t* sides, const double* pole,
                  double re, double* traction, double* loads) {
  if (nb <= 0 || ntri <= 0) return;
  LoadsK K{};
  K.g = g;
  K.bodies = bodies;
  K.nb = nb;
  K.ntri = ntri;
  K.u = u;
  K.v = v;
  K.w = w;
  K.p = p;
  K.p32 = p32;
  K.cb_mask = cb_mask;
  K.sides = sides;
  K.inv_re = 1.0 / re;
  K.traction = traction;
  IBM_LAUNCH(pf, "loads_markers", s, (k_loads_markers<<<(ntri + 63) / 64, 64, 0, s>>>(K)));
  IBM_LAUNCH(pf, "loads_sum", s, (k_loads_sum<<<nb, 256, 0, s>>>(bodies, traction, pole, loads)));
}

}  // namespace ibm
