// Direct solve of L_c phi = rhs (paper Eq. elliptic / elliptic_mod, Sec. 2:
// FFTs along the periodic directions and a tridiagonal solve along the
// wall-normal one), in five passes over HBM:
//   1. per x-row: form the right-hand side (from an array, or on the fly from
//      the predicted velocity: (D u - q_F)/(alpha dt) on C_F, 0 on C_B) and
//      transform it along x; keep the nx/2+1 non-redundant bins
//   2. per (y-plane, tile of x-modes): complex FFT along z
//   3. per mode (p, m): Thomas along y with the diagonal shifted by the
//      eigenvalues lambda_x(p) + lambda_z(m) of the periodic second
//      differences; the singular (0,0) mode has its first row replaced by
//      phi_0 = 0 and is shifted to zero volume-weighted mean
//   4. inverse z transform, 5. inverse x transform -> phi.
// The transforms are mixed-radix (2, 3, 4, 5, 7) Stockham autosort FFTs
// staged in LDS (ping-pong buffers), twiddles from a precomputed FP64 table.
#include "geom.h"

namespace ibm {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}

struct PlanDev {
  int n, nst;
  int radix[16];
  const double2* tw;
};

// small DFT of size R on u[0..R-1] (forward: exp(-2 pi i rq/R)); R is a
// compile-time constant so the butterfly stays in registers
template <int R, bool INV>
__device__ __forceinline__ void small_dft(double2* u, const double2* tw, int n) {
  if constexpr (R == 2) {
    const double2 a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const double2 a0 = u[0], a1 = u[1], a2 = u[2], a3 = u[3];
    const double2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const double2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
    // forward: multiply d13 by -i; inverse: by +i
    const double2 rot = INV ? make_double2(-d13.y, d13.x) : make_double2(d13.y, -d13.x);
    u[0] = cadd(s02, s13);
    u[1] = cadd(d02, rot);
    u[2] = csub(s02, s13);
    u[3] = csub(d02, rot);
  } else {
    double2 w[R];
    const int st = n / R;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      w[m] = tw[m * st];
      if (INV) w[m].y = -w[m].y;
    }
    double2 y[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double2 acc = u[0];
#pragma unroll
      for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(u[r], w[(r * q) % R]));
      y[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] = y[q];
  }
}

// one Stockham stage of radix R (current sub-transform length p) for ncols
// sequences at buf[idx*si + col*sc]
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(const double2* src, double2* dst, const PlanDev& P,
                                          int p, int ncols, int si, int sc) {
  const int n = P.n;
  const int T = n / R;
  const int step = n / (p * R);
  const int total = T * ncols;
  for (int bb = threadIdx.x; bb < total; bb += blockDim.x) {
    // neighbouring threads take neighbouring LDS addresses
    const int col = (si == 1) ? bb / T : bb % ncols;
    const int i = (si == 1) ? bb % T : bb / ncols;
    const int k = i % p;
    double2 u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = src[(i + r * T) * si + col * sc];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 w = P.tw[r * k * step];
      if (INV) w.y = -w.y;
      u[r] = cmul(u[r], w);
    }
    small_dft<R, INV>(u, P.tw, n);
    const int ob = (i - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(ob + r * p) * si + col * sc] = u[r];
  }
}

// Stockham FFT of ncols independent length-n sequences held in LDS at
// buf[idx*si + col*sc]; ping-pongs between a and b; returns the buffer that
// holds the result.  All threads of the block must call it.
template <bool INV>
__device__ double2* lds_fft(double2* a, double2* b, const PlanDev& P, int ncols, int si, int sc) {
  int p = 1;
  double2* src = a;
  double2* dst = b;
  for (int s = 0; s < P.nst; ++s) {
    const int R = P.radix[s];
    switch (R) {
      case 2: fft_stage<2, INV>(src, dst, P, p, ncols, si, sc); break;
      case 3: fft_stage<3, INV>(src, dst, P, p, ncols, si, sc); break;
      case 4: fft_stage<4, INV>(src, dst, P, p, ncols, si, sc); break;
      case 5: fft_stage<5, INV>(src, dst, P, p, ncols, si, sc); break;
      default: fft_stage<7, INV>(src, dst, P, p, ncols, si, sc); break;
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
    p *= R;
  }
  return src;
}

struct PoisK {
  GridView g;
  PlanDev px, pz;
  const double* rhs;
  const double *u, *v, *w;
  const uint32_t* cb_mask;
  const double* qf;
  double inv_adt;
  double2* spec;
  double* cscr;
  const double* lamx;
  const double* lamz;
  const double* ylo;
  const double* yhi;
  double inv_sum_dy;
  double scale;
  double* phi;
  int rows;  // x-rows per block
  int tp;    // x-modes per block in the z passes
};

__global__ __launch_bounds__(256) void k_fftx_fwd(PoisK K) {
  extern __shared__ double2 sm[];
  const GridView& g = K.g;
  const int nx = g.nx, nxh = g.nxh;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int64_t row0 = (int64_t)blockIdx.x * K.rows;
  const int nr = (int)((row0 + K.rows <= nrows) ? K.rows : nrows - row0);
  double2* a = sm;
  double2* b = sm + K.rows * nx;
  const int64_t plane = (int64_t)g.nz * nx;
  const double q = K.rhs ? 0.0 : *K.qf;
  for (int e = threadIdx.x; e < nr * nx; e += blockDim.x) {
    const int r = e / nx, i = e % nx;
    const int64_t cell = (row0 + r) * nx + i;
    double val;
    if (K.rhs) {
      val = K.rhs[cell];
    } else if (K.cb_mask && test_bit(K.cb_mask, cell)) {
      val = 0.0;
    } else {
      const int64_t rr = row0 + r;
      const int j = (int)(rr / g.nz), k = (int)(rr % g.nz);
      const int ip = (i + 1 == nx) ? 0 : i + 1;
      const int kp = (k + 1 == g.nz) ? 0 : k + 1;
      const double D = (K.u[cell - i + ip] - K.u[cell]) * g.idx +
                       (K.v[cell + plane] - K.v[cell]) * g.idy[j] +
                       (K.w[(int64_t)j * plane + (int64_t)kp * nx + i] - K.w[cell]) * g.idz;
      val = (D - q) * K.inv_adt;
    }
    a[r * nx + i] = make_double2(val, 0.0);
  }
  for (int e = nr * nx + threadIdx.x; e < K.rows * nx; e += blockDim.x)
    a[e] = make_double2(0.0, 0.0);
  __syncthreads();
  double2* out = lds_fft<false>(a, b, K.px, K.rows, 1, nx);
  for (int e = threadIdx.x; e < nr * nxh; e += blockDim.x) {
    const int r = e / nxh, p = e % nxh;
    K.spec[(row0 + r) * nxh + p] = out[r * nx + p];
  }
}

template <bool INV>
__global__ __launch_bounds__(256) void k_fftz(PoisK K) {
  extern __shared__ double2 sm[];
  const GridView& g = K.g;
  const int nz = g.nz, nxh = g.nxh, tp = K.tp;
  const int j = blockIdx.y;
  const int p0 = blockIdx.x * tp;
  const int nc = (p0 + tp <= nxh) ? tp : nxh - p0;
  double2* a = sm;
  double2* b = sm + nz * tp;
  double2* spec = K.spec + (int64_t)j * nz * nxh + p0;
  for (int e = threadIdx.x; e < nz * tp; e += blockDim.x) {
    const int k = e / tp, c = e % tp;
    a[e] = (c < nc) ? spec[(int64_t)k * nxh + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  double2* out = lds_fft<INV>(a, b, K.pz, tp, tp, 1);
  for (int e = threadIdx.x; e < nz * tp; e += blockDim.x) {
    const int k = e / tp, c = e % tp;
    if (c < nc) spec[(int64_t)k * nxh + c] = out[e];
  }
}

constexpr int YCH = 4;

__global__ __launch_bounds__(256) void k_tri_y(PoisK K) {
  const GridView& g = K.g;
  const int nxh = g.nxh;
  const int64_t nm = (int64_t)g.nz * nxh;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nm) return;
  const int m = (int)(q / nxh), p = (int)(q % nxh);
  const double lam = K.lamx[p] + K.lamz[m];
  const int ny = g.ny;
  double2* __restrict__ X = K.spec + q;
  double* __restrict__ C = K.cscr + q;
  const bool zero = (q == 0);
  double cpp = 0.0;
  double2 dpp = make_double2(0.0, 0.0);
  for (int j0 = 0; j0 < ny; j0 += YCH) {
    double2 buf[YCH];
#pragma unroll
    for (int t = 0; t < YCH; ++t)
      if (j0 + t < ny) buf[t] = X[(int64_t)(j0 + t) * nm];
#pragma unroll
    for (int t = 0; t < YCH; ++t) {
      const int j = j0 + t;
      if (j < ny) {
        double a = K.ylo[j], c = K.yhi[j], b = lam - (a + c);
        double2 d = buf[t];
        if (zero && j == 0) {
          a = 0.0;
          b = 1.0;
          c = 0.0;
          d = make_double2(0.0, 0.0);
        }
        const double mm = 1.0 / (b - a * cpp);
        const double cp = c * mm;
        const double2 dp = make_double2((d.x - a * dpp.x) * mm, (d.y - a * dpp.y) * mm);
        C[(int64_t)j * nm] = cp;
        buf[t] = dp;
        cpp = cp;
        dpp = dp;
      }
    }
#pragma unroll
    for (int t = 0; t < YCH; ++t)
      if (j0 + t < ny) X[(int64_t)(j0 + t) * nm] = buf[t];
  }
  double2 xn = make_double2(0.0, 0.0);
  double2 msum = make_double2(0.0, 0.0);
  for (int j1 = ny; j1 > 0; j1 -= YCH) {
    double2 buf[YCH];
    double cb[YCH];
#pragma unroll
    for (int t = 0; t < YCH; ++t)
      if (j1 - 1 - t >= 0) {
        buf[t] = X[(int64_t)(j1 - 1 - t) * nm];
        cb[t] = C[(int64_t)(j1 - 1 - t) * nm];
      }
#pragma unroll
    for (int t = 0; t < YCH; ++t) {
      const int j = j1 - 1 - t;
      if (j >= 0) {
        const double2 x = make_double2(buf[t].x - cb[t] * xn.x, buf[t].y - cb[t] * xn.y);
        buf[t] = x;
        xn = x;
        if (zero) {
          msum.x += g.dy[j] * x.x;
          msum.y += g.dy[j] * x.y;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < YCH; ++t)
      if (j1 - 1 - t >= 0) X[(int64_t)(j1 - 1 - t) * nm] = buf[t];
  }
  if (zero) {  // zero volume-weighted mean of phi
    const double2 M = make_double2(msum.x * K.inv_sum_dy, msum.y * K.inv_sum_dy);
    for (int j = 0; j < ny; ++j) X[(int64_t)j * nm] = csub(X[(int64_t)j * nm], M);
  }
}

__global__ __launch_bounds__(256) void k_fftx_inv(PoisK K) {
  extern __shared__ double2 sm[];
  const GridView& g = K.g;
  const int nx = g.nx, nxh = g.nxh;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int64_t row0 = (int64_t)blockIdx.x * K.rows;
  const int nr = (int)((row0 + K.rows <= nrows) ? K.rows : nrows - row0);
  double2* a = sm;
  double2* b = sm + K.rows * nx;
  for (int e = threadIdx.x; e < K.rows * nx; e += blockDim.x) {
    const int r = e / nx, i = e % nx;
    double2 val = make_double2(0.0, 0.0);
    if (r < nr) {
      if (i < nxh) {
        val = K.spec[(row0 + r) * nxh + i];
      } else {  // Hermitian extension of a real sequence
        const double2 c = K.spec[(row0 + r) * nxh + (nx - i)];
        val = make_double2(c.x, -c.y);
      }
    }
    a[e] = val;
  }
  __syncthreads();
  double2* out = lds_fft<true>(a, b, K.px, K.rows, 1, nx);
  for (int e = threadIdx.x; e < nr * nx; e += blockDim.x)
    K.phi[row0 * nx + e] = out[e].x * K.scale;
}

static PlanDev to_dev(const FFTPlan* p) {
  PlanDev d;
  d.n = p->n;
  d.nst = p->nst;
  for (int i = 0; i < 16; ++i) d.radix[i] = p->radix[i];
  d.tw = p->tw;
  return d;
}

void launch_poisson(Prof* pf, hipStream_t s, const GridView& g, const PoissonArgs& a,
                    const double* rhs, const double* u, const double* v, const double* w,
                    const uint32_t* cb_mask, const double* qf, double inv_adt, double* phi) {
  PoisK K{};
  K.g = g;
  K.px = to_dev(a.px);
  K.pz = to_dev(a.pz);
  K.rhs = rhs;
  K.u = u;
  K.v = v;
  K.w = w;
  K.cb_mask = cb_mask;
  K.qf = qf;
  K.inv_adt = inv_adt;
  K.spec = a.spec;
  K.cscr = a.cscr;
  K.lamx = a.lamx;
  K.lamz = a.lamz;
  K.ylo = a.ylo;
  K.yhi = a.yhi;
  K.inv_sum_dy = 1.0 / a.sum_dy;
  K.scale = 1.0 / ((double)g.nx * g.nz);
  K.phi = phi;
  int rows = 2048 / g.nx;
  if (rows < 1) rows = 1;
  if (rows > 8) rows = 8;
  K.rows = rows;
  int tp = 2048 / g.nz;
  if (tp < 1) tp = 1;
  if (tp > 8) tp = 8;
  K.tp = tp;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int xblocks = (int)((nrows + rows - 1) / rows);
  const size_t xsh = 2 * (size_t)rows * g.nx * sizeof(double2);
  const size_t zsh = 2 * (size_t)tp * g.nz * sizeof(double2);
  const int xthreads = 256;
  dim3 zgrid((g.nxh + tp - 1) / tp, g.ny);
  const int64_t nm = (int64_t)g.nz * g.nxh;
  IBM_LAUNCH(pf, "pois_fftx_fwd", s, k_fftx_fwd<<<xblocks, xthreads, xsh, s>>>(K));
  IBM_LAUNCH(pf, "pois_fftz_fwd", s, k_fftz<false><<<zgrid, 256, zsh, s>>>(K));
  IBM_LAUNCH(pf, "pois_tri_y", s, k_tri_y<<<(int)((nm + 255) / 256), 256, 0, s>>>(K));
  IBM_LAUNCH(pf, "pois_fftz_inv", s, k_fftz<true><<<zgrid, 256, zsh, s>>>(K));
  IBM_LAUNCH(pf, "pois_fftx_inv", s, k_fftx_inv<<<xblocks, xthreads, xsh, s>>>(K));
}

}  // namespace ibm
