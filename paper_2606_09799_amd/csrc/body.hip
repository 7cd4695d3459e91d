// Vertex positions and velocities at t^n from host-evaluated coefficients
// (the wall position X(t) and velocity U(X(t)) of the problem statement,
// Sec. 2).  Only +, - and * in a fixed order, without contraction into FMA,
// so that the vertices (and hence the tags) are bit-identical to any other
// implementation of the same order.
#pragma clang fp contract(off)

#include "lanes.h"

namespace ibm {

struct Rigid {
  double c[3], R[9], cd[3], om[3];
};
struct Deform {
  double c[3], r0, s, sd, cd[3];
};

// X = c + R X0, U = cdot + omega x (X - c)
__device__ __forceinline__ void rigid_vertex(const Rigid& k, const double* __restrict__ x0, int v,
                                             double* __restrict__ xyz, double* __restrict__ vel) {
  double a0 = x0[3 * v], a1 = x0[3 * v + 1], a2 = x0[3 * v + 2];
  double X[3];
  for (int d = 0; d < 3; ++d)
    X[d] = k.c[d] + ((k.R[3 * d] * a0 + k.R[3 * d + 1] * a1) + k.R[3 * d + 2] * a2);
  double r0 = X[0] - k.c[0], r1 = X[1] - k.c[1], r2 = X[2] - k.c[2];
  xyz[3 * v] = X[0];
  xyz[3 * v + 1] = X[1];
  xyz[3 * v + 2] = X[2];
  vel[3 * v] = k.cd[0] + (k.om[1] * r2 - k.om[2] * r1);
  vel[3 * v + 1] = k.cd[1] + (k.om[2] * r0 - k.om[0] * r2);
  vel[3 * v + 2] = k.cd[2] + (k.om[0] * r1 - k.om[1] * r0);
}

// X = c + (r0 + f s) d, U = cdot + (f sdot) d (the shape carried by a
// centre moving at cdot)
__device__ __forceinline__ void deform_vertex(const Deform& k, const double* __restrict__ data,
                                              int v, double* __restrict__ xyz,
                                              double* __restrict__ vel) {
  double f = data[4 * v + 3];
  double rad = k.r0 + f * k.s;
  double rd = f * k.sd;
  for (int d = 0; d < 3; ++d) {
    double dir = data[4 * v + d];
    xyz[3 * v + d] = k.c[d] + rad * dir;
    vel[3 * v + d] = k.cd[d] + rd * dir;
  }
}

__global__ void k_body_rigid(const double* __restrict__ x0, int nv, Rigid k,
                             double* __restrict__ xyz, double* __restrict__ vel) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  rigid_vertex(k, x0, v, xyz, vel);
}

__global__ void k_body_deform(const double* __restrict__ data, int nv, Deform k,
                              double* __restrict__ xyz, double* __restrict__ vel) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  deform_vertex(k, data, v, xyz, vel);
}

// the same transforms with the coefficients read from device memory (the
// layout of the host coefficient vectors), so that a captured launch can be
// replayed with new coefficients
struct BodyRigidDevK {
  const double* x0;
  int nv;
  const double* coef;
  double* xyz;
  double* vel;
};
template <bool G = false>
__global__ void k_body_rigid_dev(GArg<BodyRigidDevK, G> grp_arg_) {
  uint3 bid, gdim;
  const BodyRigidDevK& P_ = grp_enter<BodyRigidDevK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  const double* __restrict__ x0 = P_.x0;
  int nv = P_.nv;
  const double* __restrict__ coef = P_.coef;
  double* __restrict__ xyz = P_.xyz;
  double* __restrict__ vel = P_.vel;
  int v = bid.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  Rigid k;
  for (int d = 0; d < 3; ++d) k.c[d] = coef[d];
  for (int d = 0; d < 9; ++d) k.R[d] = coef[3 + d];
  for (int d = 0; d < 3; ++d) k.cd[d] = coef[12 + d];
  for (int d = 0; d < 3; ++d) k.om[d] = coef[15 + d];
  rigid_vertex(k, x0, v, xyz, vel);
}

struct BodyDeformDevK {
  const double* data;
  int nv;
  const double* coef;
  double* xyz;
  double* vel;
};
template <bool G = false>
__global__ void k_body_deform_dev(GArg<BodyDeformDevK, G> grp_arg_) {
  uint3 bid, gdim;
  const BodyDeformDevK& P_ = grp_enter<BodyDeformDevK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  const double* __restrict__ data = P_.data;
  int nv = P_.nv;
  const double* __restrict__ coef = P_.coef;
  double* __restrict__ xyz = P_.xyz;
  double* __restrict__ vel = P_.vel;
  int v = bid.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  Deform k;
  for (int d = 0; d < 3; ++d) k.c[d] = coef[d];
  k.r0 = coef[3];
  k.s = coef[4];
  k.sd = coef[5];
  for (int d = 0; d < 3; ++d) k.cd[d] = coef[6 + d];
  deform_vertex(k, data, v, xyz, vel);
}

void launch_body_rigid(Prof* pf, hipStream_t s, const double* x0, int nv, const double* coef,
                       double* xyz, double* vel) {
  Rigid k;
  for (int d = 0; d < 3; ++d) k.c[d] = coef[d];
  for (int d = 0; d < 9; ++d) k.R[d] = coef[3 + d];
  for (int d = 0; d < 3; ++d) k.cd[d] = coef[12 + d];
  for (int d = 0; d < 3; ++d) k.om[d] = coef[15 + d];
  if (nv <= 0) return;
  IBM_LAUNCH(pf, "body_rigid", s,
             k_body_rigid<<<(nv + 255) / 256, 256, 0, s>>>(x0, nv, k, xyz, vel));
}

void launch_body_deform(Prof* pf, hipStream_t s, const double* data, int nv, const double* coef,
                        double* xyz, double* vel) {
  Deform k;
  for (int d = 0; d < 3; ++d) k.c[d] = coef[d];
  k.r0 = coef[3];
  k.s = coef[4];
  k.sd = coef[5];
  for (int d = 0; d < 3; ++d) k.cd[d] = coef[6 + d];
  if (nv <= 0) return;
  IBM_LAUNCH(pf, "body_deform", s,
             k_body_deform<<<(nv + 255) / 256, 256, 0, s>>>(data, nv, k, xyz, vel));
}

void launch_body_dev(Prof* pf, hipStream_t s, int deform, const double* ref, int nv,
                     const double* coef_dev, double* xyz, double* vel) {
  if (nv <= 0) return;
  const dim3 grid((unsigned)((nv + 255) / 256));
  if (deform) {
    const BodyDeformDevK K{ref, nv, coef_dev, xyz, vel};
    IBM_LAUNCH_G(pf, "body_deform", s, (&k_body_deform_dev<true>), grid, dim3(256), 0, K,
                 k_body_deform_dev<<<grid, 256, 0, s>>>(K));
  } else {
    const BodyRigidDevK K{ref, nv, coef_dev, xyz, vel};
    IBM_LAUNCH_G(pf, "body_rigid", s, (&k_body_rigid_dev<true>), grid, dim3(256), 0, K,
                 k_body_rigid_dev<<<grid, 256, 0, s>>>(K));
  }
}

}  // namespace ibm
