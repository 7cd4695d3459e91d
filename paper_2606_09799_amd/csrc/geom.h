// Device geometry shared by the tagging and forcing kernels: the closest
// point of a triangle to a point (the fast point-triangle algorithm the paper
// cites for Alg. 1: Ericson, Real-Time Collision Detection, 2004, Sec. 5.1.5,
// Voronoi regions of vertices, edges and face tested in that order) and the
// description of the three staggered lattices.
//
// Arithmetic contract: only IEEE binary64 +, -, *, / in the written order,
// never contracted into FMA (this header and its includers are compiled with
// contraction off), so that every implementation of the same order obtains
// the same bits.
#pragma once
#pragma clang fp contract(off)

#include "lanes.h"

namespace ibm {

__device__ __forceinline__ double dot3(double a0, double a1, double a2, double b0, double b1,
                                       double b2) {
  return (a0 * b0 + a1 * b1) + a2 * b2;
}

struct ClosestPt {
  double x[3];  // closest point
  double w[3];  // barycentric weights on (A, B, C)
};

__device__ inline ClosestPt closest_point(const double p[3], const double A[3],
                                          const double B[3], const double C[3]) {
  ClosestPt r;
  const double ab0 = B[0] - A[0], ab1 = B[1] - A[1], ab2 = B[2] - A[2];
  const double ac0 = C[0] - A[0], ac1 = C[1] - A[1], ac2 = C[2] - A[2];
  const double ap0 = p[0] - A[0], ap1 = p[1] - A[1], ap2 = p[2] - A[2];
  const double d1 = dot3(ab0, ab1, ab2, ap0, ap1, ap2);
  const double d2 = dot3(ac0, ac1, ac2, ap0, ap1, ap2);
  if (d1 <= 0.0 && d2 <= 0.0) {  // vertex A
    r.x[0] = A[0]; r.x[1] = A[1]; r.x[2] = A[2];
    r.w[0] = 1.0; r.w[1] = 0.0; r.w[2] = 0.0;
    return r;
  }
  const double bp0 = p[0] - B[0], bp1 = p[1] - B[1], bp2 = p[2] - B[2];
  const double d3 = dot3(ab0, ab1, ab2, bp0, bp1, bp2);
  const double d4 = dot3(ac0, ac1, ac2, bp0, bp1, bp2);
  if (d3 >= 0.0 && d4 <= d3) {  // vertex B
    r.x[0] = B[0]; r.x[1] = B[1]; r.x[2] = B[2];
    r.w[0] = 0.0; r.w[1] = 1.0; r.w[2] = 0.0;
    return r;
  }
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {  // edge AB
    const double t = d1 / (d1 - d3);
    r.x[0] = A[0] + ab0 * t; r.x[1] = A[1] + ab1 * t; r.x[2] = A[2] + ab2 * t;
    r.w[0] = 1.0 - t; r.w[1] = t; r.w[2] = 0.0;
    return r;
  }
  const double cp0 = p[0] - C[0], cp1 = p[1] - C[1], cp2 = p[2] - C[2];
  const double d5 = dot3(ab0, ab1, ab2, cp0, cp1, cp2);
  const double d6 = dot3(ac0, ac1, ac2, cp0, cp1, cp2);
  if (d6 >= 0.0 && d5 <= d6) {  // vertex C
    r.x[0] = C[0]; r.x[1] = C[1]; r.x[2] = C[2];
    r.w[0] = 0.0; r.w[1] = 0.0; r.w[2] = 1.0;
    return r;
  }
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {  // edge AC
    const double t = d2 / (d2 - d6);
    r.x[0] = A[0] + ac0 * t; r.x[1] = A[1] + ac1 * t; r.x[2] = A[2] + ac2 * t;
    r.w[0] = 1.0 - t; r.w[1] = 0.0; r.w[2] = t;
    return r;
  }
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {  // edge BC
    const double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    r.x[0] = B[0] + (C[0] - B[0]) * t;
    r.x[1] = B[1] + (C[1] - B[1]) * t;
    r.x[2] = B[2] + (C[2] - B[2]) * t;
    r.w[0] = 0.0; r.w[1] = 1.0 - t; r.w[2] = t;
    return r;
  }
  const double den = 1.0 / ((va + vb) + vc);  // face
  const double s = vb * den, t = vc * den;
  r.x[0] = (A[0] + ab0 * s) + ac0 * t;
  r.x[1] = (A[1] + ab1 * s) + ac1 * t;
  r.x[2] = (A[2] + ab2 * s) + ac2 * t;
  r.w[0] = (1.0 - s) - t; r.w[1] = s; r.w[2] = t;
  return r;
}

// The staggered lattice of velocity component c (0 = u, 1 = v, 2 = w):
// x offset ox, z offset oz (cell units) and the y heights including the two
// wall points; valid (unknown) nodes are ext indices e_first..e_last.
struct Lattice {
  double ox, oz;
  const double* ext;
  int next, e_first, e_last;
};

__device__ __forceinline__ Lattice lattice(const GridView& g, int c) {
  Lattice L;
  L.ox = (c == 0) ? 0.0 : 0.5;
  L.oz = (c == 2) ? 0.0 : 0.5;
  if (c == 1) {
    L.ext = g.yf;
    L.next = g.ny + 1;
    L.e_first = 1;
    L.e_last = g.ny - 1;
  } else {
    L.ext = g.extuw;
    L.next = g.ny + 2;
    L.e_first = 1;
    L.e_last = g.ny;
  }
  return L;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// first index with ext[i] >= v (numpy searchsorted side='left')
__device__ __forceinline__ int lower_bound(const double* ext, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (ext[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}
// first index with ext[i] > v (side='right')
__device__ __forceinline__ int upper_bound(const double* ext, int n, double v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (ext[mid] <= v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int find_body(const BodyDev* b, int nbody, int t) {
  int k = 0;
  while (k + 1 < nbody && t >= b[k + 1].toff) ++k;
  return k;
}

// Candidate node-index box of a triangle on lattice c: the nodes inside its
// bounding box inflated by the largest neighbour spacing, plus one node of
// margin on each side (x and z unwrapped, y clamped to the valid nodes).
struct Box {
  int i0, i1, e0, e1, k0, k1;
};

__device__ __forceinline__ Box candidate_box(const GridView& g, const Lattice& L,
                                             const double lo[3], const double hi[3]) {
  const double dm = g.dmax;
  Box b;
  b.i0 = (int)floor((lo[0] - dm) / g.dx - L.ox) - 1;
  b.i1 = (int)floor((hi[0] + dm) / g.dx - L.ox) + 1;
  b.k0 = (int)floor((lo[2] - dm) / g.dz - L.oz) - 1;
  b.k1 = (int)floor((hi[2] + dm) / g.dz - L.oz) + 1;
  int e0 = lower_bound(L.ext, L.next, lo[1] - dm) - 1;
  int e1 = upper_bound(L.ext, L.next, hi[1] + dm);
  b.e0 = e0 < L.e_first ? L.e_first : (e0 > L.e_last ? L.e_last : e0);
  b.e1 = e1 < L.e_first ? L.e_first : (e1 > L.e_last ? L.e_last : e1);
  return b;
}

__device__ __forceinline__ void load_triangle(const BodyDev* bodies, int nbody, int t,
                                              double A[3], double B[3], double C[3],
                                              const double** vel, int vid[3]) {
  const BodyDev& bd = bodies[find_body(bodies, nbody, t)];
  const int lt = t - bd.toff;
  vid[0] = bd.tri[3 * lt];
  vid[1] = bd.tri[3 * lt + 1];
  vid[2] = bd.tri[3 * lt + 2];
  for (int d = 0; d < 3; ++d) {
    A[d] = bd.xyz[3 * vid[0] + d];
    B[d] = bd.xyz[3 * vid[1] + d];
    C[d] = bd.xyz[3 * vid[2] + d];
  }
  *vel = bd.vel;
}

}  // namespace ibm
