// Explicit right-hand side of the predictor (paper Eq. NS_prov in delta form):
//   R = dt [gamma H(u) + rho H_prev - alpha (G p - f) + (alpha/Re) L u]
// on the fluid nodes, R = 0 on the forcing nodes (Eq. IB_step: those nodes
// are not predicted) and on the v wall planes.  H = -div(u u) in flux
// (conservative) form; L the viscous Laplacian with the wall value 0 at half
// a cell from the first centre; G p the staggered pressure gradient; f the
// constant driving force along x.
//
// One thread per (i, j, k) computes the three components; x is the fastest
// thread index so every neighbour access of a wavefront is a contiguous row
// segment.  The neighbourhood reuse across rows is served by the L2: tiles
// are ordered so that each XCD sweeps a contiguous slab (xcd_tile).
//
// Storage type T of p, H and R: double, or float in the mixed form.  The
// stencil arithmetic is FP64 in both forms: the velocity is FP64, and
// rounding it to FP32 before differencing would amplify its rounding error by
// 1/spacing; only the results are stored in T.
#include "geom.h"

namespace ibm {

template <typename T>
struct RhsK {
  GridView g;
  const double *u, *v, *w;
  const T* p;
  const T* hprev[3];
  T* hout[3];
  T* R[3];
  const uint32_t* mask[3];
  double gamma, rho, alpha, dt, re, fx;
};

#define IDX(i, j, k) (((int64_t)(j) * g.nz + (k)) * g.nx + (i))

template <typename T>
__global__ __launch_bounds__(256) void k_rhs(RhsK<T> K) {
  const GridView& g = K.g;
  const RhsK<T>& a = K;
  const int nbx = (g.nx + 63) / 64, nbz = (g.nz + 3) / 4;
  const int64_t t = xcd_tile(blockIdx.x, (int64_t)nbx * nbz * g.ny);
  const int i = (int)(t % nbx) * 64 + threadIdx.x;
  const int k = (int)((t / nbx) % nbz) * 4 + threadIdx.y;
  const int j = (int)(t / ((int64_t)nbx * nbz));
  if (i >= g.nx || k >= g.nz) return;
  const int im = (i == 0) ? g.nx - 1 : i - 1;
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int km = (k == 0) ? g.nz - 1 : k - 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const double idx = g.idx, idz = g.idz;
  const double idx2 = idx * idx, idz2 = idz * idz;
  const double* __restrict__ u = a.u;
  const double* __restrict__ v = a.v;
  const double* __restrict__ w = a.w;
  const T* __restrict__ p = a.p;
  const int64_t c = IDX(i, j, k);
  const double idyj = g.idy[j];
  const bool has_s = j > 0, has_n = j + 1 < g.ny;
  const double ic_n = g.idyc[j + 1], ic_s = g.idyc[j];
  // weights of the face interpolations at faces j+1 (north) and j (south)
  const double n0 = g.fw0[j + 1], n1 = g.fw1[j + 1], s0 = g.fw0[j], s1 = g.fw1[j];
  const double am = a.alpha / a.re;

  // ------------------------------------------------------------ u node
  {
    const double uc = u[c], ue = u[IDX(ip, j, k)], uw = u[IDX(im, j, k)];
    const double ut = u[IDX(i, j, kp)], ub = u[IDX(i, j, km)];
    const double un = has_n ? u[IDX(i, j + 1, k)] : 0.0;
    const double us = has_s ? u[IDX(i, j - 1, k)] : 0.0;
    const double bp = 0.5 * (uc + ue), bm = 0.5 * (uw + uc);
    const double tx = (bp * bp - bm * bm) * idx;
    const double iyn = has_n ? uc * n0 + un * n1 : 0.0;
    const double iys = has_s ? us * s0 + uc * s1 : 0.0;
    const double vn = 0.5 * (v[IDX(im, j + 1, k)] + v[IDX(i, j + 1, k)]);
    const double vs = 0.5 * (v[IDX(im, j, k)] + v[IDX(i, j, k)]);
    const double ty = (iyn * vn - iys * vs) * idyj;
    const double fzp = (0.5 * (uc + ut)) * (0.5 * (w[IDX(im, j, kp)] + w[IDX(i, j, kp)]));
    const double fzm = (0.5 * (ub + uc)) * (0.5 * (w[IDX(im, j, k)] + w[IDX(i, j, k)]));
    const double tz = (fzp - fzm) * idz;
    const double H = -(tx + ty + tz);
    const double L = ((ue - uc) - (uc - uw)) * idx2 + ((ut - uc) - (uc - ub)) * idz2 +
                     ((un - uc) * ic_n - (uc - us) * ic_s) * idyj;
    const double gp = ((double)p[c] - (double)p[IDX(im, j, k)]) * idx;
    double r = a.gamma * H - a.alpha * (gp - a.fx) + am * L;
    if (a.rho != 0.0) r += a.rho * (double)a.hprev[0][c];
    if (a.hout[0]) a.hout[0][c] = (T)H;
    a.R[0][c] = (T)(test_bit(a.mask[0], c) ? 0.0 : a.dt * r);
  }
  // ------------------------------------------------------------ w node
  {
    const double wc = w[c], we = w[IDX(ip, j, k)], ww = w[IDX(im, j, k)];
    const double wt = w[IDX(i, j, kp)], wb = w[IDX(i, j, km)];
    const double wn = has_n ? w[IDX(i, j + 1, k)] : 0.0;
    const double ws = has_s ? w[IDX(i, j - 1, k)] : 0.0;
    const double bp = 0.5 * (wc + wt), bm = 0.5 * (wb + wc);
    const double tz = (bp * bp - bm * bm) * idz;
    const double iyn = has_n ? wc * n0 + wn * n1 : 0.0;
    const double iys = has_s ? ws * s0 + wc * s1 : 0.0;
    const double vn = 0.5 * (v[IDX(i, j + 1, km)] + v[IDX(i, j + 1, k)]);
    const double vs = 0.5 * (v[IDX(i, j, km)] + v[IDX(i, j, k)]);
    const double ty = (iyn * vn - iys * vs) * idyj;
    const double fxp = (0.5 * (wc + we)) * (0.5 * (u[IDX(ip, j, km)] + u[IDX(ip, j, k)]));
    const double fxm = (0.5 * (ww + wc)) * (0.5 * (u[IDX(i, j, km)] + u[IDX(i, j, k)]));
    const double tx = (fxp - fxm) * idx;
    const double H = -(tx + ty + tz);
    const double L = ((we - wc) - (wc - ww)) * idx2 + ((wt - wc) - (wc - wb)) * idz2 +
                     ((wn - wc) * ic_n - (wc - ws) * ic_s) * idyj;
    const double gp = ((double)p[c] - (double)p[IDX(i, j, km)]) * idz;
    double r = a.gamma * H - a.alpha * gp + am * L;
    if (a.rho != 0.0) r += a.rho * (double)a.hprev[2][c];
    if (a.hout[2]) a.hout[2][c] = (T)H;
    a.R[2][c] = (T)(test_bit(a.mask[2], c) ? 0.0 : a.dt * r);
  }
  // ------------------------------------------------------ v node (face j)
  if (j == 0) {
    a.R[1][c] = (T)0;  // wall planes
    a.R[1][IDX(i, g.ny, k)] = (T)0;
    if (a.hout[1]) {
      a.hout[1][c] = (T)0;
      a.hout[1][IDX(i, g.ny, k)] = (T)0;
    }
    return;
  }
  {
    const double vc = v[c], ve = v[IDX(ip, j, k)], vw = v[IDX(im, j, k)];
    const double vt = v[IDX(i, j, kp)], vb = v[IDX(i, j, km)];
    const double vn = v[IDX(i, j + 1, k)], vs = v[IDX(i, j - 1, k)];
    const double uy_i = u[IDX(i, j - 1, k)] * s0 + u[c] * s1;
    const double uy_ip = u[IDX(ip, j - 1, k)] * s0 + u[IDX(ip, j, k)] * s1;
    const double tx = (uy_ip * (0.5 * (vc + ve)) - uy_i * (0.5 * (vw + vc))) * idx;
    const double ct = 0.5 * (vc + vn), cs = 0.5 * (vs + vc);
    const double ty = (ct * ct - cs * cs) * ic_s;
    const double wy_k = w[IDX(i, j - 1, k)] * s0 + w[c] * s1;
    const double wy_kp = w[IDX(i, j - 1, kp)] * s0 + w[IDX(i, j, kp)] * s1;
    const double tz = (wy_kp * (0.5 * (vc + vt)) - wy_k * (0.5 * (vb + vc))) * idz;
    const double H = -(tx + ty + tz);
    const double L = ((ve - vc) - (vc - vw)) * idx2 + ((vt - vc) - (vc - vb)) * idz2 +
                     ((vn - vc) * idyj - (vc - vs) * g.idy[j - 1]) * ic_s;
    const double gp = ((double)p[c] - (double)p[IDX(i, j - 1, k)]) * ic_s;
    double r = a.gamma * H - a.alpha * gp + am * L;
    if (a.rho != 0.0) r += a.rho * (double)a.hprev[1][c];
    if (a.hout[1]) a.hout[1][c] = (T)H;
    a.R[1][c] = (T)(test_bit(a.mask[1], c) ? 0.0 : a.dt * r);
  }
}

template <typename T>
static void run_rhs(Prof* pf, hipStream_t s, const GridView& g, const RhsArgs& a) {
  RhsK<T> K;
  K.g = g;
  K.u = a.u;
  K.v = a.v;
  K.w = a.w;
  K.p = static_cast<const T*>(a.p);
  for (int q = 0; q < 3; ++q) {
    K.hprev[q] = static_cast<const T*>(a.hprev[q]);
    K.hout[q] = static_cast<T*>(a.hout[q]);
    K.R[q] = static_cast<T*>(a.R[q]);
    K.mask[q] = a.mask[q];
  }
  K.gamma = a.gamma;
  K.rho = a.rho;
  K.alpha = a.alpha;
  K.dt = a.dt;
  K.re = a.re;
  K.fx = a.fx;
  dim3 block(64, 4);
  const int64_t tiles = (int64_t)((g.nx + 63) / 64) * ((g.nz + 3) / 4) * g.ny;
  dim3 grid((unsigned)tiles);
  IBM_LAUNCH(pf, "rhs", s, k_rhs<T><<<grid, block, 0, s>>>(K));
}

void launch_rhs(Prof* pf, hipStream_t s, const GridView& g, const RhsArgs& a) {
  if (a.fp32)
    run_rhs<float>(pf, s, g, a);
  else
    run_rhs<double>(pf, s, g, a);
}

}  // namespace ibm
