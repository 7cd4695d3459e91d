// Projection and pressure update (paper Eqs. projection and update_pressure):
//   u <- u_hat - alpha dt G phi   on every interior velocity node
//   p <- p + phi - alpha dt/(2 Re) L_c phi,  L_c = D G (Neumann at the walls)
// One thread per (i, j, k), x fastest; blocks of 256 x-points of one row in
// the XCD band order (xcd_band_tile: bands of 16 rows, walked plane by
// plane), so that the rows of phi at k-1, k+1 and the planes j-1, j+1 are
// reused from the same L2.  Rows shorter than 256 points go 256/nx rows
// (consecutive k) to a block, so that its threads are not left idle.  The velocity update is FP64 in both forms; p is
// stored in T (float in the mixed form) and updated in FP64 arithmetic.
#include "lanes.h"

namespace ibm {

constexpr int PROJ_BAND = 16;  // rows per band of the block order

template <typename T>
struct ProjK {
  GridView g;
  const double* phi;
  double adt, pc;
  double *u, *v, *w;
  T* p;
  int rpb;  // rows per block: 256/nx for rows shorter than 256, else 1
  int bw;   // rows (of blocks) per band: PROJ_BAND, fewer on small planes
};

template <typename T, bool G = false>
__global__ __launch_bounds__(256) void k_project(GArg<ProjK<T>, G> grp_arg_) {
  uint3 bid, gdim;
  const ProjK<T>& P_ = grp_enter<ProjK<T>, G>(grp_arg_, bid, gdim);
  const GridView& g = P_.g;
  const double* __restrict__ phi = P_.phi;
  const double adt = P_.adt, pc = P_.pc;
  double* __restrict__ u = P_.u;
  double* __restrict__ v = P_.v;
  double* __restrict__ w = P_.w;
  T* __restrict__ p = P_.p;
  const int R = P_.rpb;
  const int nbx = (R > 1) ? 1 : (g.nx + 255) / 256;
  const int nbz = (g.nz + R - 1) / R;
  int it, kb, j;
  if (!xcd_band_tile(bid.x, nbx, nbz, g.ny, P_.bw, it, kb, j)) return;
  int i, k;
  if (R > 1) {
    const int r = (int)threadIdx.x / g.nx;
    i = (int)threadIdx.x - r * g.nx;
    k = kb * R + r;
    if (r >= R || k >= g.nz) return;
  } else {
    i = it * 256 + threadIdx.x;
    k = kb;
    if (i >= g.nx) return;
  }
  const int64_t plane = (int64_t)g.nz * g.nx;
  const int64_t c = (int64_t)j * plane + (int64_t)k * g.nx + i;
  const int im = (i == 0) ? g.nx - 1 : i - 1;
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int km = (k == 0) ? g.nz - 1 : k - 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const int64_t row = (int64_t)j * plane + (int64_t)k * g.nx;
  const double fc = phi[c];
  const double fw = phi[row + im], fe = phi[row + ip];
  const double fb = phi[(int64_t)j * plane + (int64_t)km * g.nx + i];
  const double ft = phi[(int64_t)j * plane + (int64_t)kp * g.nx + i];
  const double gx = (fc - fw) * g.idx;
  const double gz = (fc - fb) * g.idz;
  u[c] -= adt * gx;
  w[c] -= adt * gz;
  double fluxs = 0.0, fluxn = 0.0;
  if (j > 0) {
    const double gy = (fc - phi[c - plane]) * g.idyc[j];
    v[c] -= adt * gy;
    fluxs = gy;
  }
  if (j + 1 < g.ny) fluxn = (phi[c + plane] - fc) * g.idyc[j + 1];
  const double lc = ((fe - fc) * g.idx - gx) * g.idx + ((ft - fc) * g.idz - gz) * g.idz +
                    (fluxn - fluxs) * g.idy[j];
  p[c] = (T)((double)p[c] + (fc - pc * lc));
}

void launch_project(Prof* pf, hipStream_t s, const GridView& g, const double* phi, double adt,
                    double re, double* u, double* v, double* w, void* p, int fp32) {
  const int rpb = (g.nx < 256) ? 256 / g.nx : 1;
  const int nbx = (rpb > 1) ? 1 : (g.nx + 255) / 256;
  const int nbz = (g.nz + rpb - 1) / rpb;
  // bands of PROJ_BAND rows; on planes of fewer than 8 such bands, narrower
  // ones (the padding of the last band round would otherwise be most blocks)
  int bw = nbz / 8;
  bw = bw < 1 ? 1 : (bw > PROJ_BAND ? PROJ_BAND : bw);
  dim3 grid((unsigned)xcd_band_blocks(nbx, nbz, g.ny, bw));
  const double pc = adt / (2.0 * re);
  if (fp32) {
    const ProjK<float> K{g, phi, adt, pc, u, v, w, (float*)p, rpb, bw};
    IBM_LAUNCH_G(pf, "project", s, (&k_project<float, true>), grid, dim3(256), 0, K,
                 k_project<float><<<grid, 256, 0, s>>>(K));
  } else {
    const ProjK<double> K{g, phi, adt, pc, u, v, w, (double*)p, rpb, bw};
    IBM_LAUNCH_G(pf, "project", s, (&k_project<double, true>), grid, dim3(256), 0, K,
                 k_project<double><<<grid, 256, 0, s>>>(K));
  }
}

}  // namespace ibm
