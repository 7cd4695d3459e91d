// Rigid-body dynamics of the loosely coupled FSI (paper Sec. 4.5, with the
// loads of Sec. 3.3): one thread per body advances Newton's equations (the
// fluid force plus an external force, inertial frame), Euler's equations
// (principal frame, torque about the body's centre brought in by R^T) and
// the unit quaternion dq/dt = q (x) (0, Omega)/2 by AB2 (explicit Euler on
// the first step), renormalises q, and writes the 18 coefficients of the
// rigid motion at the new time (c, R row-major, cdot, omega in the world
// frame) that the body transform reads from device memory.
#include "ibm.h"
#include "lanes.h"

namespace ibm {

__device__ __forceinline__ void quat_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

__global__ void k_rigid_advance(int nb, double* __restrict__ state, const double* __restrict__ props,
                                const double* __restrict__ loads, double dt,
                                double* __restrict__ coef) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  double* s = state + (int64_t)b * IBM_RIGID_STATE;
  const double* pr = props + (int64_t)b * IBM_RIGID_PROPS;
  const double* ld = loads + 6 * (int64_t)b;
  double c[3], q[4], V[3], Om[3];
  for (int d = 0; d < 3; ++d) {
    c[d] = s[d];
    V[d] = s[7 + d];
    Om[d] = s[10 + d];
  }
  for (int d = 0; d < 4; ++d) q[d] = s[3 + d];
  const double m = pr[0], I[3] = {pr[1], pr[2], pr[3]};
  double R[9];
  quat_rot(q, R);
  // derivatives now: dV, dOm, dc, dq
  double dv[13];
  for (int d = 0; d < 3; ++d) dv[d] = (ld[d] + pr[4 + d]) / m;
  double Mb[3], IOm[3] = {I[0] * Om[0], I[1] * Om[1], I[2] * Om[2]};
  for (int a = 0; a < 3; ++a) Mb[a] = R[a] * ld[3] + R[3 + a] * ld[4] + R[6 + a] * ld[5];
  const double cr[3] = {Om[1] * IOm[2] - Om[2] * IOm[1], Om[2] * IOm[0] - Om[0] * IOm[2],
                        Om[0] * IOm[1] - Om[1] * IOm[0]};
  for (int a = 0; a < 3; ++a) dv[3 + a] = (Mb[a] - cr[a]) / I[a];
  for (int d = 0; d < 3; ++d) dv[6 + d] = V[d];
  // q (x) (0, Om)
  dv[9] = 0.5 * (-q[1] * Om[0] - q[2] * Om[1] - q[3] * Om[2]);
  dv[10] = 0.5 * (q[0] * Om[0] + q[2] * Om[2] - q[3] * Om[1]);
  dv[11] = 0.5 * (q[0] * Om[1] - q[1] * Om[2] + q[3] * Om[0]);
  dv[12] = 0.5 * (q[0] * Om[2] + q[1] * Om[1] - q[2] * Om[0]);
  const bool started = s[26] != 0.0;
  double inc[13];
  for (int a = 0; a < 13; ++a) inc[a] = dt * (started ? 1.5 * dv[a] - 0.5 * s[13 + a] : dv[a]);
  for (int d = 0; d < 3; ++d) {
    s[7 + d] = V[d] + inc[d];
    s[10 + d] = Om[d] + inc[3 + d];
    s[d] = c[d] + inc[6 + d];
  }
  double qn[4], n2 = 0.0;
  for (int d = 0; d < 4; ++d) {
    qn[d] = q[d] + inc[9 + d];
    n2 += qn[d] * qn[d];
  }
  const double nq = sqrt(n2);
  for (int d = 0; d < 4; ++d) s[3 + d] = qn[d] / nq;
  for (int a = 0; a < 13; ++a) s[13 + a] = dv[a];
  s[26] = 1.0;
  double Rn[9], qq[4] = {s[3], s[4], s[5], s[6]};
  quat_rot(qq, Rn);
  double* co = coef + (int64_t)b * 18;
  for (int d = 0; d < 3; ++d) co[d] = s[d];
  for (int d = 0; d < 9; ++d) co[3 + d] = Rn[d];
  for (int d = 0; d < 3; ++d) co[12 + d] = s[7 + d];
  for (int a = 0; a < 3; ++a)
    co[15 + a] = Rn[3 * a] * s[10] + Rn[3 * a + 1] * s[11] + Rn[3 * a + 2] * s[12];
}

void launch_rigid_advance(Prof* pf, hipStream_t s, int nb, double* state, const double* props,
                          const double* loads, double dt, double* coef) {
  if (nb <= 0) return;
  IBM_LAUNCH(pf, "rigid_advance", s,
             (k_rigid_advance<<<(nb + 63) / 64, 64, 0, s>>>(nb, state, props, loads, dt, coef)));
}

}  // namespace ibm
