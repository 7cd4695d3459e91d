// Direct solve of L_c phi = rhs (paper Eq. elliptic / elliptic_mod, Sec. 2:
// FFTs along the periodic directions and a tridiagonal solve along the
// wall-normal one), in five passes over HBM:
//   1. per x-row: form the right-hand side (from an array, or on the fly from
//      the predicted velocity: (D u - q_F)/(alpha dt) on C_F, 0 on C_B) and
//      transform it along x; keep the nx/2+1 non-redundant bins
//   2. per (y-plane, tile of x-modes): complex FFT along z
//   3. per mode (p, m): tridiagonal solve along y with the diagonal shifted by
//      the eigenvalues lambda_x(p) + lambda_z(m) of the periodic second
//      differences; the singular (0,0) mode has its first row replaced by
//      phi_0 = 0 and is shifted to zero volume-weighted mean
//   4. inverse z transform, 5. inverse x transform -> phi.
// The transforms are mixed-radix (2, 3, 4, 5, 7) Stockham autosort FFTs
// staged in LDS (ping-pong buffers), twiddles from a precomputed table; the
// real x transforms carry two rows per complex sequence.
//
// Spectral precision.  The spectrum and the transforms are FP64 (double2) or
// FP32 (float2, the mixed form).  The wall-normal solves always run in FP64
// arithmetic.  In the mixed form the FP32 solve S is the inner solver of an
// FP64-residual refinement: phi = S(rhs), then while max|rhs - L_c phi| is
// above the tolerance, phi += S(rhs - L_c phi).  The residual is formed in
// FP64 inside the first pass of the next solve; the decision to go on is
// taken on the device (every pass of a refinement returns at once when the
// residual that opened it is below the tolerance), so the whole sequence is
// enqueued without any host synchronisation.
#include "lanes.h"

namespace ibm {

template <typename C> struct RealOf;
template <> struct RealOf<double2> { using T = double; };
template <> struct RealOf<float2> { using T = float; };

template <typename C>
__device__ __forceinline__ C mkc(typename RealOf<C>::T a, typename RealOf<C>::T b) {
  C r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return mkc<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
  return mkc<C>(a.x + b.x, a.y + b.y);
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
  return mkc<C>(a.x - b.x, a.y - b.y);
}

template <typename C>
struct PlanDev {
  int n, nst;
  int radix[16];
  const C* tw;
};

// small DFT of size R on u[0..R-1] (forward: exp(-2 pi i rq/R)); R is a
// compile-time constant so the butterfly stays in registers
template <typename C, int R, bool INV>
__device__ __forceinline__ void small_dft(C* u, const C* tw, int n) {
  if constexpr (R == 2) {
    const C a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const C a0 = u[0], a1 = u[1], a2 = u[2], a3 = u[3];
    const C s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const C s13 = cadd(a1, a3), d13 = csub(a1, a3);
    // forward: multiply d13 by -i; inverse: by +i
    const C rot = INV ? mkc<C>(-d13.y, d13.x) : mkc<C>(d13.y, -d13.x);
    u[0] = cadd(s02, s13);
    u[1] = cadd(d02, rot);
    u[2] = csub(s02, s13);
    u[3] = csub(d02, rot);
  } else {
    C w[R];
    const int st = n / R;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      w[m] = tw[m * st];
      if (INV) w[m].y = -w[m].y;
    }
    C y[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      C acc = u[0];
#pragma unroll
      for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(u[r], w[(r * q) % R]));
      y[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] = y[q];
  }
}

// Transforms hold at most 32 KB of LDS per block (two ping-pong buffers of
// fft_buf complex values each), so that four blocks share a CU.
template <typename C>
constexpr int fft_buf() { return 16384 / (int)sizeof(C); }

// one Stockham stage of radix R (current sub-transform length p) for ncols
// sequences at buf[idx*si + col*sc]
template <typename C, int R, bool INV>
__device__ __forceinline__ void fft_stage(const C* src, C* dst, const PlanDev<C>& P, int p,
                                          int ncols, int si, int sc) {
  const int n = P.n;
  const int T = n / R;
  const int step = n / (p * R);
  const int total = T * ncols;
  for (int bb = threadIdx.x; bb < total; bb += blockDim.x) {
    // neighbouring threads take neighbouring LDS addresses
    const int col = (si == 1) ? bb / T : bb % ncols;
    const int i = (si == 1) ? bb % T : bb / ncols;
    const int k = i % p;
    C u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = src[(i + r * T) * si + col * sc];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      C w = P.tw[r * k * step];
      if (INV) w.y = -w.y;
      u[r] = cmul(u[r], w);
    }
    small_dft<C, R, INV>(u, P.tw, n);
    const int ob = (i - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(ob + r * p) * si + col * sc] = u[r];
  }
}

// Stockham FFT of ncols independent length-n sequences held in LDS at
// buf[idx*si + col*sc]; ping-pongs between a and b; returns the buffer that
// holds the result.  All threads of the block must call it.
template <typename C, bool INV>
__device__ C* lds_fft(C* a, C* b, const PlanDev<C>& P, int ncols, int si, int sc) {
  int p = 1;
  C* src = a;
  C* dst = b;
  for (int s = 0; s < P.nst; ++s) {
    const int R = P.radix[s];
    switch (R) {
      case 2: fft_stage<C, 2, INV>(src, dst, P, p, ncols, si, sc); break;
      case 3: fft_stage<C, 3, INV>(src, dst, P, p, ncols, si, sc); break;
      case 4: fft_stage<C, 4, INV>(src, dst, P, p, ncols, si, sc); break;
      case 5: fft_stage<C, 5, INV>(src, dst, P, p, ncols, si, sc); break;
      default: fft_stage<C, 7, INV>(src, dst, P, p, ncols, si, sc); break;
    }
    __syncthreads();
    C* t = src;
    src = dst;
    dst = t;
    p *= R;
  }
  return src;
}

// source of the first x pass
enum : int { SRC_ARRAY = 0, SRC_VELOCITY = 1, SRC_RESIDUAL = 2, SRC_CHECK = 3 };

template <typename C>
struct PoisK {
  GridView g;
  PlanDev<C> px, pz;
  int mode;
  const double* rhs;           // SRC_ARRAY: the right-hand side; SRC_RESIDUAL/CHECK: kept copy
  const double *u, *v, *w;     // SRC_VELOCITY
  const uint32_t* cb_mask;
  const double* qf;            // q_F, or (c0, c1) of the energy-conserving shape
  const void* pq;              // energy-conserving shape: p (else NULL)
  int pq32;                    // p stored in FP32
  double inv_adt;
  double* rhs_keep;            // FP64 copy of the right-hand side formed in pass 1 (or NULL)
  const double* phi_in;        // SRC_RESIDUAL/CHECK: current phi
  u64* rmax;                   // SRC_RESIDUAL/CHECK: max |r| (bits of a non-negative double)
  const u64* gate;             // the launch does nothing when *gate <= gate_tol
  double gate_tol;
  C* spec;
  const double* lamx;
  const double* lamz;
  const double* ylo;
  const double* yhi;
  double inv_sum_dy;
  double scale;
  double* phi;
  int accumulate;              // inverse x pass: phi += result instead of phi = result
  double* zm;                  // FP32 spectrum: the (0,0) mode column kept in FP64 (ny)
  double* psum;                // SRC_RESIDUAL: per-block sums of phi dV (fixed order)
  const double* msum;          // inverse x pass of a refinement: sum of phi dV to remove
  double inv_vtot;
  int ldx;                     // row stride of the spectrum (spec_ld)
  // wall-normal solve output: a spectrum of another precision (the FP64
  // spectrum of the refined mixed form, read by FP64 inverse passes) with its
  // own row stride; NULL: in place in spec
  void* spec_out;
  int ldx_out;
  // FP32 spectrum: the (0,0) mode's right-hand side loses its volume-weighted
  // mean before the gauged solve (see the wall-normal solves)
  int zero_in;
  int rows;                    // x-rows per block
  int tp;                      // x-modes per block in the z passes
  int yP, yL, yr, ytl;         // wall-normal solve: segments, base length, longer ones, lines per block
  int yPP;                     // yP rounded up to a power of two (lanes per mode in the reduction)
};

template <typename C>
__device__ __forceinline__ bool gated(const PoisK<C>& K) {
  return K.gate && __longlong_as_double((long long)*K.gate) <= K.gate_tol;
}

// L_c phi at one cell: the discrete operator the solve inverts (second
// differences in x and z, face fluxes in y with zero flux at the walls)
__device__ __forceinline__ double lap_c(const GridView& g, const double* __restrict__ f,
                                        int64_t cell, int i, int j, int k) {
  const int64_t plane = (int64_t)g.nz * g.nx;
  const int64_t row = cell - i;
  const int im = (i == 0) ? g.nx - 1 : i - 1;
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int km = (k == 0) ? g.nz - 1 : k - 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const double fc = f[cell];
  const double gx0 = (fc - f[row + im]) * g.idx, gx1 = (f[row + ip] - fc) * g.idx;
  const double gz0 = (fc - f[cell + (int64_t)(km - k) * g.nx]) * g.idz;
  const double gz1 = (f[cell + (int64_t)(kp - k) * g.nx] - fc) * g.idz;
  const double fs = (j > 0) ? (fc - f[cell - plane]) * g.idyc[j] : 0.0;
  const double fn = (j + 1 < g.ny) ? (f[cell + plane] - fc) * g.idyc[j + 1] : 0.0;
  return (gx1 - gx0) * g.idx + (gz1 - gz0) * g.idz + (fn - fs) * g.idy[j];
}

// Right-hand side of the solve at cell i of x-row rr = j nz + k (the caller
// supplies j and k), by source mode; the residual modes also accumulate
// max|r| and phi dV, and the FP64 copy is kept when asked.  q, q1: q_F, or
// (c0, c1) of the energy shape.
template <typename C>
__device__ __forceinline__ double fftx_source(const PoisK<C>& K, int64_t rr, int j, int k, int i,
                                              double q, double q1, double& rmax, double& vsum) {
  const GridView& g = K.g;
  const int nx = g.nx;
  const int64_t plane = (int64_t)g.nz * nx;
  const int64_t cell = rr * nx + i;
  double val;
  if (K.mode == SRC_ARRAY) {
    val = K.rhs[cell];
  } else if (K.mode == SRC_VELOCITY) {
    if (K.cb_mask && test_bit(K.cb_mask, cell)) {
      val = 0.0;
    } else {
      const int ip = (i + 1 == nx) ? 0 : i + 1;
      const int kp = (k + 1 == g.nz) ? 0 : k + 1;
      const double u0 = K.u[cell], u1 = K.u[cell - i + ip];
      const double v0 = K.v[cell], v1 = K.v[cell + plane];
      const double w0 = K.w[cell], w1 = K.w[(int64_t)j * plane + (int64_t)kp * nx + i];
      const double D = (u1 - u0) * g.idx + (v1 - v0) * g.idy[j] + (w1 - w0) * g.idz;
      double qq = q;
      if (K.pq) {  // q_F = c0 + c1 (p - e), e the cell's kinetic energy
        const double eu = 0.5 * (u0 * u0 + u1 * u1);
        const double ev = 0.5 * (v0 * v0 + v1 * v1);
        const double ew = 0.5 * (w0 * w0 + w1 * w1);
        const double pc = K.pq32 ? (double)static_cast<const float*>(K.pq)[cell]
                                 : static_cast<const double*>(K.pq)[cell];
        qq = q + q1 * (pc - 0.5 * ((eu + ev) + ew));
      }
      val = (D - qq) * K.inv_adt;
    }
  } else {
    val = K.rhs[cell] - lap_c(g, K.phi_in, cell, i, j, k);
    rmax = fmax(rmax, fabs(val));
    vsum += K.phi_in[cell] * g.dy[j];
  }
  if (K.rhs_keep) K.rhs_keep[cell] = val;
  return val;
}

// block maximum of |r| (one atomic on its bit pattern: non-negative doubles
// order like their bits) and block sum of phi dV into psum[bx] (bx: the
// block's index in its launch), in a fixed order; red: 2 * (waves per block)
// doubles of LDS
__device__ __forceinline__ void resid_reduce(double rmax, double vsum, double* red, u64* rmax_out,
                                             double* psum, double dxdz, uint32_t bx) {
  for (int off = 32; off > 0; off >>= 1) {
    rmax = fmax(rmax, __shfl_xor(rmax, off));
    vsum += __shfl_xor(vsum, off);
  }
  const int nw = (int)(blockDim.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = rmax;
    red[nw + (threadIdx.x >> 6)] = vsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0], sm = red[nw];
    for (int t = 1; t < nw; ++t) {
      m = fmax(m, red[t]);
      sm += red[nw + t];
    }
    atomicMax(reinterpret_cast<unsigned long long*>(rmax_out),
              (unsigned long long)__double_as_longlong(m));
    if (psum) psum[bx] = sm * dxdz;
  }
}

// Velocity source (SRC_VELOCITY without the energy shape) of the generic
// forward x transform on rows of nx = 256 M values, 256 threads: thread t
// forms x = t + 256 m (m < M) of each row, all loads issued whatever the C_B
// mask says (same arithmetic as fftx_source), so that a row's loads are in
// flight together.  Rows past nr take the block's first row, stored as 0.
template <typename C, bool CB, int M>
__device__ __forceinline__ void fftx_stage_vel_rows(const PoisK<C>& K, typename RealOf<C>::T* sr,
                                                    int64_t row0, int nr, int rows, double q) {
  using R = typename RealOf<C>::T;
  const GridView& g = K.g;
  constexpr int nx = 256 * M;
  const int nz = g.nz;
  const int64_t plane = (int64_t)nz * nx;
#pragma unroll 2
  for (int r = 0; r < rows; ++r) {
    const int64_t rr = row0 + (r < nr ? r : 0);
    const int jr = (int)(rr / nz), kr = (int)(rr - (int64_t)jr * nz);
    const int kp = (kr + 1 == nz) ? 0 : kr + 1;
    const double idyj = g.idy[jr];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int i = (int)threadIdx.x + 256 * m;
      const int ip = (i + 1 == nx) ? 0 : i + 1;
      const int64_t cell = rr * nx + i;
      const double u0 = K.u[cell], u1 = K.u[cell - i + ip];
      const double v0 = K.v[cell], v1 = K.v[cell + plane];
      const double w0 = K.w[cell], w1 = K.w[(int64_t)jr * plane + (int64_t)kp * nx + i];
      const double D = (u1 - u0) * g.idx + (v1 - v0) * idyj + (w1 - w0) * g.idz;
      double val = (D - q) * K.inv_adt;
      if (CB && ((K.cb_mask[cell >> 5] >> (uint32_t)(cell & 31)) & 1u)) val = 0.0;
      if (r >= nr) val = 0.0;
      sr[2 * ((r >> 1) * nx + i) + (r & 1)] = (R)val;
    }
  }
}

template <typename C, bool G = false>
__global__ __launch_bounds__(256) void k_fftx_fwd(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using R = typename RealOf<C>::T;
  if (gated(K)) return;
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  __shared__ double red[8];
  const GridView& g = K.g;
  const int nx = g.nx, nxh = g.nxh;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int64_t row0 = (int64_t)bid.x * K.rows;
  const int nr = (int)((row0 + K.rows <= nrows) ? K.rows : nrows - row0);
  // two real rows per complex sequence: row r is the real (r even) or the
  // imaginary (r odd) part of sequence r/2
  R* sr = reinterpret_cast<R*>(sm);
  const double q = (K.mode == SRC_VELOCITY) ? K.qf[0] : 0.0;
  const double q1 = (K.mode == SRC_VELOCITY && K.pq) ? K.qf[1] : 0.0;
  const bool resid = K.mode >= SRC_RESIDUAL;
  double rmax = 0.0, vsum = 0.0;
  const bool fast = K.mode == SRC_VELOCITY && !K.rhs_keep && !K.pq && blockDim.x == 256 &&
                    (nx == 512 || nx == 1024);
  if (fast) {  // every row of the block staged, rows past nr as 0
    if (nx == 512) {
      if (K.cb_mask) fftx_stage_vel_rows<C, true, 2>(K, sr, row0, nr, K.rows, q);
      else fftx_stage_vel_rows<C, false, 2>(K, sr, row0, nr, K.rows, q);
    } else {
      if (K.cb_mask) fftx_stage_vel_rows<C, true, 4>(K, sr, row0, nr, K.rows, q);
      else fftx_stage_vel_rows<C, false, 4>(K, sr, row0, nr, K.rows, q);
    }
  } else {
    for (int e = threadIdx.x; e < nr * nx; e += blockDim.x) {
      const int r = e / nx, i = e % nx;
      const int64_t rr = row0 + r;
      const int jr = (int)(rr / g.nz), kr = (int)(rr - (int64_t)jr * g.nz);
      const double val = fftx_source(K, rr, jr, kr, i, q, q1, rmax, vsum);
      if (K.mode != SRC_CHECK) sr[2 * ((r >> 1) * nx + i) + (r & 1)] = (R)val;
    }
    if (resid) {
      resid_reduce(rmax, vsum, red, K.rmax, K.psum, g.dx * g.dz, bid.x);
      if (K.mode == SRC_CHECK) return;  // block-uniform
    }
    for (int e = nr * nx + threadIdx.x; e < K.rows * nx; e += blockDim.x) {
      const int r = e / nx, i = e % nx;
      sr[2 * ((r >> 1) * nx + i) + (r & 1)] = (R)0;
    }
  }
  __syncthreads();
  const C* out = lds_fft<C, false>(sm, sm + (K.rows / 2) * nx, K.px, K.rows / 2, 1, nx);
  // split: with Z = A + iB, A[k] = (Z[k] + conj Z[n-k])/2, B[k] = (Z[k] - conj Z[n-k])/2i
  for (int e = threadIdx.x; e < nr * nxh; e += blockDim.x) {
    const int r = e / nxh, p = e % nxh;
    const C zk = out[(r >> 1) * nx + p];
    const C zm = out[(r >> 1) * nx + (p == 0 ? 0 : nx - p)];
    const R h = (R)0.5;
    K.spec[(row0 + r) * K.ldx + p] = (r & 1) ? mkc<C>(h * (zk.y + zm.y), h * (zm.x - zk.x))
                                           : mkc<C>(h * (zk.x + zm.x), h * (zk.y - zm.y));
  }
}

template <typename C, bool INV, bool G = false>
__global__ __launch_bounds__(256) void k_fftz(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using R = typename RealOf<C>::T;
  if (gated(K)) return;
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  const GridView& g = K.g;
  const int nz = g.nz, nxh = g.nxh, tp = K.tp;
  const int j = bid.y;
  const int p0 = bid.x * tp;
  const int nc = (p0 + tp <= nxh) ? tp : nxh - p0;
  C* spec = K.spec + (int64_t)j * nz * K.ldx + p0;
  for (int e = threadIdx.x; e < nz * tp; e += blockDim.x) {
    const int k = e / tp, c = e % tp;
    sm[e] = (c < nc) ? spec[(int64_t)k * K.ldx + c] : mkc<C>((R)0, (R)0);
  }
  __syncthreads();
  const C* out = lds_fft<C, INV>(sm, sm + nz * tp, K.pz, tp, tp, 1);
  for (int e = threadIdx.x; e < nz * tp; e += blockDim.x) {
    const int k = e / tp, c = e % tp;
    if (c < nc) spec[(int64_t)k * K.ldx + c] = out[e];
  }
}

// ---------------------------------------------------------------------------
// Length-256 transforms as 16 x 16 (four-step): a thread loads 16 values of
// its sequence (stride 16) from HBM, takes a 16-point DFT in registers
// (radix 4 x 4), multiplies by the twiddles W_256^(n1 k2) and writes them
// transposed to LDS; after one barrier each thread takes the second
// 16-point DFT over the other index and stores its 16 outputs.  One LDS
// round trip and one barrier instead of a Stockham stage per radix-4 factor.

// forward: exp(-2 pi i m/16); inverse: the conjugate (m a compile-time value
// in the unrolled loops below)
template <typename C, bool INV>
__device__ __forceinline__ C w16(int m) {
  using R = typename RealOf<C>::T;
  const double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
  const double r2 = 0.70710678118654752440;
  const double cs[16] = {1, c1, r2, s1, 0, -s1, -r2, -c1, -1, -c1, -r2, -s1, 0, s1, r2, c1};
  const double sn = cs[(m + 12) & 15];  // sin(2 pi m/16) = cos(2 pi (m - 4)/16)
  return mkc<C>((R)cs[m & 15], (R)(INV ? sn : -sn));
}

template <typename C, bool INV>
__device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  const C s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const C s13 = cadd(a1, a3), d13 = csub(a1, a3);
  // forward: -i d13; inverse: +i d13
  const C rot = INV ? mkc<C>(-d13.y, d13.x) : mkc<C>(d13.y, -d13.x);
  a0 = cadd(s02, s13);
  a1 = cadd(d02, rot);
  a2 = csub(s02, s13);
  a3 = csub(d02, rot);
}

// 16-point DFT in place; output k = k1 + 4 k2 is left at x[4 k1 + k2]
template <typename C, bool INV>
__device__ __forceinline__ void dft16(C (&x)[16]) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<C, INV>(x[n2], x[n2 + 4], x[n2 + 8], x[n2 + 12]);
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) x[n2 + 4 * k1] = cmul(x[n2 + 4 * k1], w16<C, INV>(n2 * k1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<C, INV>(x[4 * k1], x[4 * k1 + 1], x[4 * k1 + 2], x[4 * k1 + 3]);
}
__device__ __forceinline__ constexpr int pos16(int k) { return 4 * (k & 3) + (k >> 2); }

constexpr int Z16_TC = 8;                  // x-modes per block
constexpr int Z16_LP = 16 * Z16_TC + 8;    // padded LDS stride of one k2 group

template <typename C, bool INV, bool G = false>
__global__ __launch_bounds__(16 * Z16_TC) void k_fftz256(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  if (gated(K)) return;
  __shared__ C T[16 * Z16_LP];
  const GridView& g = K.g;
  const int nxh = g.nxh;
  const int c = threadIdx.x % Z16_TC, t = threadIdx.x / Z16_TC;
  const int p = bid.x * Z16_TC + c;
  const bool valid = p < nxh;
  const int ldx = K.ldx;
  C* col = K.spec + (int64_t)bid.y * 256 * ldx + (valid ? p : 0);  // element k at col[k * ldx]
  C x[16];
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) x[n2] = col[(int64_t)(t + 16 * n2) * ldx];
  dft16<C, INV>(x);
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    C w = K.pz.tw[t * k2];
    if (INV) w.y = -w.y;
    T[k2 * Z16_LP + t * Z16_TC + c] = (k2 && t) ? cmul(x[pos16(k2)], w) : x[pos16(k2)];
  }
  __syncthreads();
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) x[n1] = T[t * Z16_LP + n1 * Z16_TC + c];
  dft16<C, INV>(x);
  if (valid) {
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) col[(int64_t)(t + 16 * k1) * ldx] = x[pos16(k1)];
  }
}

// Length 256 R z transforms (R = 2, 4: lengths 512 and 1024) as 16 x 16 x R
// (four-step twice).  With M = 16 R threads per mode (t = 0..M-1) and
// n = t + M n2:
//  1. thread t loads x[t + M n2], n2 = 0..15, from HBM, takes a 16-point DFT
//     (output k2) and the twiddle W_n^(t k2), and writes it to LDS;
//  2. thread (k2, t1) (t = t1 + R t2) reads the 16 values t2 of its k2,
//     takes a 16-point DFT (output k3) and the twiddle W_M^(t1 k3), and
//     writes them back to LDS;
//  3. each thread takes 16/R of the length-R DFTs over t1 (output k4) and
//     stores X[k2 + 16 k3 + 256 k4].
// 16/R modes per block (the 256 threads of a block load 64- or 128-byte row
// pieces).  The LDS layouts keep every 16 consecutive lanes on distinct
// 16-byte bank groups: step 2 reads stride-R rows, step 3 reads an XOR
// swizzle of the (t1, mode) index by t1 of the reading thread.
// XCD-aware order of those blocks: the G tiles of TC modes that share one
// 128-byte line of a spectrum row go to one XCD, one after the other (blocks
// are dealt to the 8 XCDs round robin by linear id), so that the line is
// fetched from HBM once into that XCD's L2 instead of once per tile.  1-D
// grid of zline_blocks blocks (bx: the block's index); false for the padding
// blocks.
__device__ __forceinline__ bool zline_tile(uint32_t bx, int G, int gx, int ny, int& tile, int& j) {
  const int64_t b = bx;
  const int u = (int)((b / NUM_XCD) % G);
  const int64_t U = (b / (NUM_XCD * (int64_t)G)) * NUM_XCD + b % NUM_XCD;  // line group
  const int LG = (gx + G - 1) / G;
  if (U >= (int64_t)ny * LG) return false;
  j = (int)(U / LG);
  tile = (int)(U % LG) * G + u;
  return tile < gx;
}
static int64_t zline_blocks(int G, int gx, int ny) {
  const int64_t units = (int64_t)ny * ((gx + G - 1) / G);
  return (units + NUM_XCD - 1) / NUM_XCD * NUM_XCD * G;
}
template <typename C, int TC>
constexpr int zline_group() {
  return (128 / (TC * (int)sizeof(C))) > 1 ? 128 / (TC * (int)sizeof(C)) : 1;
}

template <typename C, bool INV, int R, bool G = false>
__global__ __launch_bounds__(256) void k_fftz4s(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  constexpr int M = 16 * R;    // threads per mode
  constexpr int N = 16 * M;    // transform length
  constexpr int TC = 256 / M;  // modes per block
  static_assert(R * TC == 16 && N * TC == 4096, "16 x 16 x R layout");
  if (gated(K)) return;
  __shared__ C T[4096];
  const GridView& g = K.g;
  const int nxh = g.nxh;
  int tile, j;
  if (!zline_tile(bid.x, zline_group<C, TC>(), (nxh + TC - 1) / TC, g.ny, tile, j)) return;
  const int c = threadIdx.x % TC, tt = threadIdx.x / TC;
  const int p = tile * TC + c;
  const bool valid = p < nxh;
  const int ldx = K.ldx;
  C* col = K.spec + (int64_t)j * N * ldx + (valid ? p : 0);  // element k at col[k ldx]
  C x[16];
  // 1.
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) x[n2] = col[(int64_t)(tt + M * n2) * ldx];
  dft16<C, INV>(x);
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    C w = K.pz.tw[tt * k2];
    if (INV) w.y = -w.y;
    T[(k2 * M + tt) * TC + c] = (k2 && tt) ? cmul(x[pos16(k2)], w) : x[pos16(k2)];
  }
  __syncthreads();
  // 2.
  const int k2 = tt / R, t1 = tt % R;
#pragma unroll
  for (int t2 = 0; t2 < 16; ++t2) x[t2] = T[(k2 * M + t1 + R * t2) * TC + c];
  dft16<C, INV>(x);
  __syncthreads();  // every step-2 read is done before the buffer is rewritten
  const int sw = t1 * TC;  // swizzle of the writing and of the reading thread alike
#pragma unroll
  for (int k3 = 0; k3 < 16; ++k3) {
    C w = K.pz.tw[16 * t1 * k3];  // W_M^(t1 k3)
    if (INV) w.y = -w.y;
    const C v = (k3 && t1) ? cmul(x[pos16(k3)], w) : x[pos16(k3)];
    // value (k2, k3, t1, c) at row k2 16 + k3, position (t1 TC + c) ^ (owner(k3) TC)
    T[(k2 * 16 + k3) * 16 + ((t1 * TC + c) ^ ((k3 / (16 / R)) * TC))] = v;
  }
  __syncthreads();
  // 3. k3 = t1 (16/R) + q: the length-R DFT over the R values of (k2, k3)
#pragma unroll
  for (int q = 0; q < 16 / R; ++q) {
    const int k3 = t1 * (16 / R) + q;
    C u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = T[(k2 * 16 + k3) * 16 + ((r * TC + c) ^ sw)];
    if constexpr (R == 2) {
      const C a = u[0], b = u[1];
      u[0] = cadd(a, b);
      u[1] = csub(a, b);
    } else {
      dft4<C, INV>(u[0], u[1], u[2], u[3]);
    }
    if (valid) {
#pragma unroll
      for (int k4 = 0; k4 < R; ++k4) col[(int64_t)(k2 + 16 * k3 + 256 * k4) * ldx] = u[k4];
    }
  }
}

// Length-256 x transforms, two real rows per complex sequence, X16_SC
// sequences (2 X16_SC consecutive rows) per block.  The 16 lanes of a
// sequence (lane t = n1 in the first DFT, k2 in the second) lie in one
// wavefront and own one LDS tile, so between the coalesced staging of the
// block's rows and of its results only wavefront syncs are needed.
constexpr int X16_SC = 8;
constexpr int X16_SS = 16 * 17;  // complex values per sequence tile (>= 2 * 129)
// loads per thread of the inverse pass's staging: 16 spectrum rows of at
// most X16_LDX_MAX values (the padded stride of 129 modes)
constexpr int X16_LDX_MAX = 144;
constexpr int X16_INV_NE = (2 * X16_SC * X16_LDX_MAX + 32 * X16_SC - 1) / (32 * X16_SC);

// Velocity source of the length-256 forward x transform for the block's
// rows (the SRC_VELOCITY case of fftx_source, same arithmetic): thread i
// forms value i of every row.  All loads are issued whatever the C_B mask
// says (a C_B cell's value is then selected to zero) and the uniform options
// are template arguments, so the loads of successive rows are in flight
// together instead of each row waiting first for its mask word.  PQ: 0 no
// energy shape, 1 p in FP64, 2 p in FP32.
template <typename C, bool CB, int PQ, bool KEEP>
__device__ __forceinline__ void fftx256_stage_vel(const PoisK<C>& K, typename RealOf<C>::T* tr,
                                                  int64_t row0, int nr, int j00, int k00,
                                                  double q, double q1, int ss) {
  using R = typename RealOf<C>::T;
  const GridView& g = K.g;
  constexpr int nx = 256;
  const int i = threadIdx.x, nz = g.nz;
  const int64_t plane = (int64_t)nz * nx;
  const int ip = (i + 1) & (nx - 1);
  // rows in batches of SB: every load of a batch is issued before its first
  // value is used, so a thread keeps SB rows of loads in flight (FP64
  // spectrum: 101 -> 93 us on 256x192x256 at an unchanged register count;
  // the FP32 kernel, whose refinement passes stage other sources, keeps one
  // row: two would raise its registers and lower its occupancy on every path)
  constexpr int SB = sizeof(C) == sizeof(double2) ? 2 : 1;
#pragma unroll
  for (int r0 = 0; r0 < 16; r0 += SB) {
  double U0[SB], U1[SB], V0[SB], V1[SB], W0[SB], W1[SB], IY[SB];
  uint32_t MW[SB];
  int64_t CL[SB];
#pragma unroll
  for (int t = 0; t < SB; ++t) {
    const int r = r0 + t;
    const int rv = r < nr ? r : 0;  // rows past the end: row 0 again, value discarded
    const unsigned kk = (unsigned)(k00 + rv);
    const unsigned jq = kk / (unsigned)nz;
    const int jr = j00 + (int)jq, kr = (int)(kk - jq * (unsigned)nz);
    const int kp = (kr + 1 == nz) ? 0 : kr + 1;
    const int64_t rowc = (row0 + rv) * nx;
    const int64_t cell = rowc + i;
    CL[t] = cell;
    U0[t] = K.u[cell];
    U1[t] = K.u[rowc + ip];
    V0[t] = K.v[cell];
    V1[t] = K.v[cell + plane];
    W0[t] = K.w[cell];
    W1[t] = K.w[(int64_t)jr * plane + (int64_t)kp * nx + i];
    IY[t] = g.idy[jr];
    MW[t] = CB ? K.cb_mask[cell >> 5] : 0u;
  }
#pragma unroll
  for (int t = 0; t < SB; ++t) {
    const int r = r0 + t;
    const int64_t cell = CL[t];
    const double u0 = U0[t], u1 = U1[t], v0 = V0[t], v1 = V1[t], w0 = W0[t], w1 = W1[t];
    const double D = (u1 - u0) * g.idx + (v1 - v0) * IY[t] + (w1 - w0) * g.idz;
    double qq = q;
    if (PQ) {
      const double eu = 0.5 * (u0 * u0 + u1 * u1);
      const double ev = 0.5 * (v0 * v0 + v1 * v1);
      const double ew = 0.5 * (w0 * w0 + w1 * w1);
      const double pc = (PQ == 2) ? (double)static_cast<const float*>(K.pq)[cell]
                                  : static_cast<const double*>(K.pq)[cell];
      qq = q + q1 * (pc - 0.5 * ((eu + ev) + ew));
    }
    double val = (D - qq) * K.inv_adt;
    if (CB && ((MW[t] >> (uint32_t)(cell & 31)) & 1u)) val = 0.0;
    // the FP64 copy a refinement reads (a template option: a global store
    // that may alias the velocity would hold back the next batch's loads)
    if (KEEP && r < nr) K.rhs_keep[cell] = val;
    if (r >= nr) val = 0.0;
    tr[2 * ((r >> 1) * ss + i) + (r & 1)] = (R)val;
  }
  }
}

// Residual source of the length-256 forward x transform (the SRC_RESIDUAL
// and SRC_CHECK cases of fftx_source, same arithmetic): r = rhs - L_c phi
// for the block's rows, thread i forming value i of every row, with max|r|
// and the sum of phi dy accumulated.  Every load of a row (rhs, phi and its
// six neighbours; at a wall the cell's own value stands in for the missing
// plane and its term is dropped afterwards) is issued before the row is
// formed.  Rows past nr take the block's first row, stored as 0.
template <typename C>
__device__ __forceinline__ void fftx256_stage_res(const PoisK<C>& K, typename RealOf<C>::T* tr,
                                                  int64_t row0, int nr, int j00, int k00,
                                                  double& rmax, double& vsum, int ss) {
  using R = typename RealOf<C>::T;
  const GridView& g = K.g;
  constexpr int nx = 256;
  const int i = threadIdx.x, nz = g.nz;
  const int64_t plane = (int64_t)nz * nx;
  const int im = (i - 1) & (nx - 1), ip = (i + 1) & (nx - 1);
  const double* __restrict__ f = K.phi_in;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int rv = r < nr ? r : 0;
    const unsigned kk = (unsigned)(k00 + rv);
    const unsigned jq = kk / (unsigned)nz;
    const int j = j00 + (int)jq, k = (int)(kk - jq * (unsigned)nz);
    const int km = (k == 0) ? nz - 1 : k - 1;
    const int kp = (k + 1 == nz) ? 0 : k + 1;
    const int64_t row = (int64_t)(row0 + rv) * nx;
    const int64_t cell = row + i;
    const bool hs = j > 0, hn = j + 1 < g.ny;
    const double b = K.rhs[cell];
    const double fc = f[cell], fw = f[row + im], fe = f[row + ip];
    const double fb = f[cell + (int64_t)(km - k) * nx], ft = f[cell + (int64_t)(kp - k) * nx];
    const double fsv = f[hs ? cell - plane : cell], fnv = f[hn ? cell + plane : cell];
    const double icj = g.idyc[j], icn = g.idyc[j + 1], iyj = g.idy[j], dyj = g.dy[j];
    const double gx0 = (fc - fw) * g.idx, gx1 = (fe - fc) * g.idx;
    const double gz0 = (fc - fb) * g.idz, gz1 = (ft - fc) * g.idz;
    const double fs = hs ? (fc - fsv) * icj : 0.0;
    const double fn = hn ? (fnv - fc) * icn : 0.0;
    const double val = b - ((gx1 - gx0) * g.idx + (gz1 - gz0) * g.idz + (fn - fs) * iyj);
    if (r < nr) {
      rmax = fmax(rmax, fabs(val));
      vsum += fc * dyj;
      if (K.rhs_keep) K.rhs_keep[cell] = val;
    }
    tr[2 * ((r >> 1) * ss + i) + (r & 1)] = (R)(r < nr ? val : 0.0);
  }
}

// the velocity staging for the uniform options of a launch
template <typename C, bool KEEP>
__device__ __forceinline__ void fftx256_stage_vel_any(const PoisK<C>& K,
                                                      typename RealOf<C>::T* tr, int64_t row0,
                                                      int nr, int j00, int k00, double q,
                                                      double q1) {
  const int pqm = K.pq ? (K.pq32 ? 2 : 1) : 0;
  if (K.cb_mask) {
    if (pqm == 0) fftx256_stage_vel<C, true, 0, KEEP>(K, tr, row0, nr, j00, k00, q, q1, X16_SS);
    else if (pqm == 1) fftx256_stage_vel<C, true, 1, KEEP>(K, tr, row0, nr, j00, k00, q, q1, X16_SS);
    else fftx256_stage_vel<C, true, 2, KEEP>(K, tr, row0, nr, j00, k00, q, q1, X16_SS);
  } else {
    if (pqm == 0) fftx256_stage_vel<C, false, 0, KEEP>(K, tr, row0, nr, j00, k00, q, q1, X16_SS);
    else if (pqm == 1) fftx256_stage_vel<C, false, 1, KEEP>(K, tr, row0, nr, j00, k00, q, q1, X16_SS);
    else fftx256_stage_vel<C, false, 2, KEEP>(K, tr, row0, nr, j00, k00, q, q1, X16_SS);
  }
}

template <typename C, bool G = false>
__global__ __launch_bounds__(32 * X16_SC) void k_fftx256_fwd(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using R = typename RealOf<C>::T;
  if (gated(K)) return;
  __shared__ C T[X16_SC * X16_SS];
  __shared__ double red[2 * (32 * X16_SC / 64)];
  const GridView& g = K.g;
  const int nxh = g.nxh;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int64_t row0 = (int64_t)bid.x * (2 * X16_SC);
  const int nr = (int)((row0 + 2 * X16_SC <= nrows) ? 2 * X16_SC : nrows - row0);
  const double q = (K.mode == SRC_VELOCITY) ? K.qf[0] : 0.0;
  const double q1 = (K.mode == SRC_VELOCITY && K.pq) ? K.qf[1] : 0.0;
  double rmax = 0.0, vsum = 0.0;
  // 1. the block's rows, coalesced: row r is the real (r even) or imaginary
  //    (r odd) part of sequence r/2, value i at T[(r/2) X16_SS + i]
  R* tr = reinterpret_cast<R*>(T);
  // (j, k) of the block's first row; the rows of a block follow in k (32-bit
  // arithmetic: ny nz < 2^31)
  const int j00 = (int)(row0 / g.nz), k00 = (int)(row0 - (int64_t)j00 * g.nz);
  static_assert(32 * X16_SC == 256 && 2 * X16_SC == 16, "one thread per x index, 16 rows");
  // (refinement passes run on FP32 spectra only; an FP64 kernel meeting one
  // takes the generic loop below)
  if (K.mode >= SRC_RESIDUAL && sizeof(C) == sizeof(float2)) {
    if constexpr (sizeof(C) == sizeof(float2))
      fftx256_stage_res<C>(K, tr, row0, nr, j00, k00, rmax, vsum, X16_SS);
  } else if (K.mode == SRC_VELOCITY && !K.rhs_keep) {
    fftx256_stage_vel_any<C, false>(K, tr, row0, nr, j00, k00, q, q1);
  } else if (K.mode == SRC_VELOCITY && sizeof(C) == sizeof(float2)) {
    // the first pass of a refined solve (FP32 spectrum) keeps its source
    if constexpr (sizeof(C) == sizeof(float2))
      fftx256_stage_vel_any<C, true>(K, tr, row0, nr, j00, k00, q, q1);
  } else
#pragma unroll 4
  for (int e = threadIdx.x; e < 2 * X16_SC * 256; e += blockDim.x) {
    const int r = e >> 8, i = e & 255;
    int kr = k00 + r, jr = j00;
    while (kr >= g.nz) {
      kr -= g.nz;
      ++jr;
    }
    const double val = (r < nr) ? fftx_source(K, row0 + r, jr, kr, i, q, q1, rmax, vsum) : 0.0;
    tr[2 * ((r >> 1) * X16_SS + i) + (r & 1)] = (R)val;
  }
  if (K.mode >= SRC_RESIDUAL) {
    resid_reduce(rmax, vsum, red, K.rmax, K.psum, g.dx * g.dz, bid.x);
    if (K.mode == SRC_CHECK) return;  // block-uniform
  }
  __syncthreads();
  // 2. the transforms: the first 16 X16_SC threads, 16 lanes per sequence
  // (the other wavefronts, which only help with the memory passes, wait at
  // the next barrier)
  if (threadIdx.x < 16 * X16_SC) {
    const int t = threadIdx.x & 15, sc = threadIdx.x >> 4;
    C* tile = T + sc * X16_SS;
    C x[16];
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) x[n2] = tile[t + 16 * n2];
    dft16<C, false>(x);
    wave_sync();
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2)
      tile[k2 * 17 + t] = (k2 && t) ? cmul(x[pos16(k2)], K.px.tw[t * k2]) : x[pos16(k2)];
    wave_sync();
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) x[n1] = tile[t * 17 + n1];
    dft16<C, false>(x);
    wave_sync();
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) tile[t + 16 * k1] = x[pos16(k1)];  // Z[k], k = t + 16 k1
    wave_sync();
    // split: with Z = A + iB, A[k] = (Z[k] + conj Z[n-k])/2,
    // B[k] = (Z[k] - conj Z[n-k])/2i; bins p = t + 16 qq of both rows
    const R h = (R)0.5;
    C A[9], B[9];
#pragma unroll
    for (int qq = 0; qq < 9; ++qq) {
      const int p = (t + 16 * qq) & 255;
      const C zk = tile[p], zm = tile[(256 - p) & 255];
      A[qq] = mkc<C>(h * (zk.x + zm.x), h * (zk.y - zm.y));
      B[qq] = mkc<C>(h * (zk.y + zm.y), h * (zm.x - zk.x));
    }
    wave_sync();
#pragma unroll
    for (int qq = 0; qq < 9; ++qq) {
      const int p = t + 16 * qq;
      if (p < nxh) {
        tile[p] = A[qq];
        tile[nxh + p] = B[qq];
      }
    }
  }
  __syncthreads();
  // 3. the block's spectrum rows (contiguous, padding included, written as 0)
  const int ldx = K.ldx;
  C* dst = K.spec + row0 * ldx;
  for (int e = threadIdx.x; e < nr * ldx; e += blockDim.x) {
    const int r = e / ldx, p = e - r * ldx;
    dst[e] = (p < nxh) ? T[(r >> 1) * X16_SS + (r & 1) * nxh + p] : mkc<C>((R)0, (R)0);
  }
}

template <typename C, bool G = false>
__global__ __launch_bounds__(32 * X16_SC) void k_fftx256_inv(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using R = typename RealOf<C>::T;
  if (gated(K)) return;
  __shared__ C T[X16_SC * X16_SS];
  const GridView& g = K.g;
  const int nxh = g.nxh;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int64_t row0 = (int64_t)bid.x * (2 * X16_SC);
  const int nr = (int)((row0 + 2 * X16_SC <= nrows) ? 2 * X16_SC : nrows - row0);
  // 1. the block's half spectra, coalesced: row r at T[(r/2) X16_SS + (r%2) nxh].
  //    The rows are contiguous in memory (padding included): every load is
  //    issued before the first LDS store, indexes past the end repeat the
  //    last value and store nothing
  const C* src = K.spec + row0 * K.ldx;
  {
    const int ldx = K.ldx, nf = nr * ldx;
    C vals[X16_INV_NE];
#pragma unroll
    for (int it = 0; it < X16_INV_NE; ++it) {
      const int f0 = threadIdx.x + it * 32 * X16_SC;
      vals[it] = src[f0 < nf ? f0 : nf - 1];
    }
#pragma unroll
    for (int it = 0; it < X16_INV_NE; ++it) {
      const int f = threadIdx.x + it * 32 * X16_SC;
      const int r = f / ldx, p = f - r * ldx;
      if (f < nf && p < nxh) T[(r >> 1) * X16_SS + (r & 1) * nxh + p] = vals[it];
    }
    if (nr < 2 * X16_SC)  // the last block: rows past the end transform zeros
      for (int e = nr * nxh + threadIdx.x; e < 2 * X16_SC * nxh; e += blockDim.x) {
        const int r = e / nxh, p = e - r * nxh;
        T[(r >> 1) * X16_SS + (r & 1) * nxh + p] = mkc<C>((R)0, (R)0);
      }
  }
  __syncthreads();
  // the transforms: the first 16 X16_SC threads, 16 lanes per sequence (the
  // other wavefronts only help with the memory passes)
  if (threadIdx.x < 16 * X16_SC) {
    const int t = threadIdx.x & 15, sc = threadIdx.x >> 4;
    C* tile = T + sc * X16_SS;
    // bin k of a half spectrum over the Hermitian extension (bins 0 and n/2 real)
    auto bin = [&](int h, int k) -> C {
      C c = (k < nxh) ? tile[h * nxh + k] : tile[h * nxh + (256 - k)];
      if (k >= nxh) c.y = -c.y;
      if (k == 0 || k == 128) c.y = (R)0;
      return c;
    };
    C x[16];
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) {
      const int k = t + 16 * n2;
      const C A = bin(0, k), B = bin(1, k);
      x[n2] = mkc<C>(A.x - B.y, A.y + B.x);  // Z = A + iB
    }
    dft16<C, true>(x);
    wave_sync();
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) {
      C w = K.px.tw[t * k2];
      w.y = -w.y;
      tile[k2 * 17 + t] = (k2 && t) ? cmul(x[pos16(k2)], w) : x[pos16(k2)];
    }
    wave_sync();
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) x[n1] = tile[t * 17 + n1];
    dft16<C, true>(x);
    wave_sync();
    // z[i], i = t + 16 k1: real part row 2 sc, imaginary part row 2 sc + 1
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) tile[t + 16 * k1] = x[pos16(k1)];
  }
  __syncthreads();
  // 2. the block's phi rows, coalesced
  const R* tr = reinterpret_cast<const R*>(T);
  const double msub = K.msum ? *K.msum * K.inv_vtot : 0.0;
  double* dst = K.phi + row0 * 256;
  for (int e = threadIdx.x; e < nr * 256; e += blockDim.x) {
    const int r = e >> 8, i = e & 255;
    double v = (double)tr[2 * ((r >> 1) * X16_SS + i) + (r & 1)] * K.scale;
    if (K.zm) v += K.zm[(int)((row0 + r) / g.nz)] * K.scale;
    v -= msub;
    if (K.accumulate)
      dst[e] += v;
    else
      dst[e] = v;
  }
}

// Inverse x transforms of length 256 R (R = 2, 4: nx = 512, 1024) as
// 16 x 16 x R, the scheme of the z transforms of those lengths, with one
// complex sequence (two real rows: Z = A + iB over the Hermitian extensions
// of their half spectra) per M = 16 R lanes of one wavefront, so that the
// three DFT stages exchange data through the sequence's own LDS tile with
// wavefront syncs only.  With n = t + M n2:
//  1. lane t loads Z[t + M n2] (n2 = 0..15) straight from the two spectrum
//     rows (64 consecutive bins per load), takes a 16-point DFT (output k2)
//     and the twiddle W_N^(t k2), and writes tile[k2][t];
//  2. lane (k2, t1) (t = t1 + R t2) reads the 16 values t2 of its k2, takes
//     a 16-point DFT (output k3) and the twiddle W_M^(t1 k3), and writes
//     tile[k2][k3 R + t1];
//  3. lane (k2, t1) takes the length-R DFTs of k3 = t1 (16/R) + q and writes
//     z[k2 + 16 k3 + 256 k4] to the tile in natural order;
//  4. the lanes store the two phi rows (real and imaginary parts of z),
//     coalesced.
// Tile rows have a stride of M + 1 complex values, so that each step's LDS
// accesses spread over all bank groups.  A sequence past the last row pair
// transforms a copy of the last rows and stores nothing.
template <typename C, int R, bool G = false>
__global__ __launch_bounds__(256) void k_fftx4s_inv(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using RT = typename RealOf<C>::T;
  constexpr int M = 16 * R;         // lanes per sequence
  constexpr int N = 16 * M;         // transform length
  constexpr int SPB = 256 / M;      // sequences per block
  constexpr int LP = M + 1;         // tile row stride
  constexpr int TS = 16 * LP;       // tile size (complex values)
  static_assert(TS >= N, "natural-order output fits the tile");
  if (gated(K)) return;
  __shared__ C T[SPB * TS];
  const GridView& g = K.g;
  const int nxh = g.nxh;  // N/2 + 1
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int t = threadIdx.x % M, sq = threadIdx.x / M;
  const int64_t ra = ((int64_t)bid.x * SPB + sq) * 2;  // rows ra (real part), ra + 1
  const bool live_a = ra < nrows, live_b = ra + 1 < nrows;
  const C* sa = K.spec + (live_a ? ra : nrows - 1) * K.ldx;
  const C* sb = K.spec + (live_b ? ra + 1 : nrows - 1) * K.ldx;
  C* tile = T + sq * TS;
  // bin k of a half spectrum over the Hermitian extension (bins 0, N/2 real)
  auto bin = [&](const C* row, int k) -> C {
    C c = row[k < nxh ? k : N - k];
    if (k >= nxh) c.y = -c.y;
    if (k == 0 || 2 * k == N) c.y = (RT)0;
    return c;
  };
  C x[16];
  // 1.
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) {
    const int k = t + M * n2;
    const C A = bin(sa, k);
    const C B = live_b ? bin(sb, k) : mkc<C>((RT)0, (RT)0);
    x[n2] = mkc<C>(A.x - B.y, A.y + B.x);
  }
  dft16<C, true>(x);
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    C w = K.px.tw[t * k2];
    w.y = -w.y;
    tile[k2 * LP + t] = (k2 && t) ? cmul(x[pos16(k2)], w) : x[pos16(k2)];
  }
  wave_sync();
  // 2.
  const int k2 = t / R, t1 = t % R;
#pragma unroll
  for (int t2 = 0; t2 < 16; ++t2) x[t2] = tile[k2 * LP + t1 + R * t2];
  dft16<C, true>(x);
  wave_sync();  // every step-2 read is done before the tile is rewritten
#pragma unroll
  for (int k3 = 0; k3 < 16; ++k3) {
    C w = K.px.tw[16 * t1 * k3];  // W_M^(t1 k3)
    w.y = -w.y;
    tile[k2 * LP + k3 * R + t1] = (k3 && t1) ? cmul(x[pos16(k3)], w) : x[pos16(k3)];
  }
  wave_sync();
  // 3.
#pragma unroll
  for (int q = 0; q < 16 / R; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) x[q * R + r] = tile[k2 * LP + (t1 * (16 / R) + q) * R + r];
  wave_sync();
#pragma unroll
  for (int q = 0; q < 16 / R; ++q) {
    C* u = x + q * R;
    if constexpr (R == 2) {
      const C a = u[0], b = u[1];
      u[0] = cadd(a, b);
      u[1] = csub(a, b);
    } else {
      dft4<C, true>(u[0], u[1], u[2], u[3]);
    }
    const int k3 = t1 * (16 / R) + q;
#pragma unroll
    for (int k4 = 0; k4 < R; ++k4) tile[k2 + 16 * k3 + 256 * k4] = u[k4];
  }
  wave_sync();
  // 4.
  const double msub = K.msum ? *K.msum * K.inv_vtot : 0.0;
  const double za = (K.zm && live_a) ? K.zm[(int)(ra / g.nz)] * K.scale : 0.0;
  const double zb = (K.zm && live_b) ? K.zm[(int)((ra + 1) / g.nz)] * K.scale : 0.0;
  double* pa = K.phi + ra * N;
#pragma unroll 4
  for (int j = 0; j < 16; ++j) {
    const int n = t + M * j;
    const C z = tile[n];
    const double va = (double)z.x * K.scale + za - msub;
    const double vb = (double)z.y * K.scale + zb - msub;
    if (live_a) {
      if (K.accumulate)
        pa[n] += va;
      else
        pa[n] = va;
    }
    if (live_b) {
      if (K.accumulate)
        pa[N + n] += vb;
      else
        pa[N + n] = vb;
    }
  }
}

// Wall-normal solves, one per Fourier mode, partitioned like the line solves
// of the predictor: each mode's ny rows are cut into P balanced segments of
// at most YL rows (6: ny = 192 gives exactly 32 separators, a power of two),
// one thread per segment, the values in registers.  Each
// thread eliminates its interior rows so that they become affine functions
// of the two separators around the segment (its own last row and the
// previous segment's), the P separator rows form a tridiagonal system solved
// by cyclic reduction, and each thread reconstructs its rows.  The separator
// rows are re-read transposed from LDS so that a mode's PP (P rounded up to a
// power of two) separators sit in consecutive lanes of one wavefront, which
// reduces them over cross-lane reads: three block barriers in all.
// Every spectral value is read once and written once; the arithmetic is FP64
// whatever the storage precision.  The systems are diagonally dominant
// (|b| >= |a| + |c|), so the elimination needs no pivoting.
constexpr int YL = 6;

// 1/x within about an ulp: the hardware reciprocal refined by two Newton
// steps (fewer instructions than the IEEE division sequence).  Used on the
// pivots of the wall-normal systems, whose magnitudes are far from the
// limits of the FP64 range.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// One step of cyclic reduction on a row kept in excess form.  A row
//   a x_minus + b x + g x_plus = d
// is stored as (a, e, g) with e = a + b + g its row sum; the diagonal is
// e - a - g.  The wall-normal systems have a, g >= 0 and e = lambda <= 0,
// and every reduction keeps that sign pattern, so the new excess
//   e' = e - k1 e_minus - k2 e_plus   (k1 = a / b_minus, k2 = g / b_plus)
// and the diagonal e' - a' - g' are sums of terms of one sign.  Formed from
// b directly they would cancel: for the low modes |b| exceeds a + g only
// by |lambda|, and near a stretched wall a + g is large, so the separator
// systems would lose up to a few hundred times the rounding of the data
// (their residual, not that of the plain elimination, sets the
// post-projection divergence of the largest grids).
__device__ __forceinline__ void excess_row(double& a, double& e, double& g, double k1, double am,
                                           double em, double k2, double gp, double ep) {
  e = e - k1 * em - k2 * ep;
  a = -am * k1;
  g = -gp * k2;
}

// SL: rows per segment (at most; 6, or 12 where 6-row segments would need
// more than 64 separators, so that a mode's separators still fit one
// wavefront).  UNI: every segment holds exactly SL rows (ny = P SL), so the
// row loops are straight-line code.
template <typename C, bool UNI, typename CO, int SL, bool G = false>
__global__ __launch_bounds__(SL == YL ? 1024 : 512) void k_tri_y(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using RO = typename RealOf<CO>::T;
  if (gated(K)) return;
  extern __shared__ __align__(16) unsigned char smraw[];
  double* sm = reinterpret_cast<double*>(smraw);  // 11 arrays [PP][TL + 1]
  const GridView& g = K.g;
  const int TL = K.ytl, P = K.yP, PP = K.yPP, SP = TL + 1;
  const int lb = threadIdx.x % TL, s = threadIdx.x / TL;
  const bool active = s < P;  // lanes of the padding segments only join the reduction
  // modes q = k ldx + p; blocks in z-major order (block b: row k = b mod nz,
  // modes p of tile b / nz), so that consecutive blocks read different z
  // rows, hence different memory channels; padding columns are skipped
  const int64_t nm = (int64_t)g.nz * K.ldx;  // stride of one y row of modes
  const int kq = (int)(bid.x % (unsigned)g.nz);
  const int pq = (int)(bid.x / (unsigned)g.nz) * TL + lb;
  const int64_t q = (int64_t)kq * K.ldx + pq;
  const bool valid = active && pq < g.nxh;
  // LDS array f, separator seg, mode lane ln (padded stride: conflict-free in
  // both the natural and the transposed order)
  auto A = [&](int f, int seg, int ln) -> double& { return sm[((size_t)f * PP + seg) * SP + ln]; };
  // Lanes of padding segments compute the last real segment's rows and lanes
  // past the last mode the last mode's system: every lane loads and solves
  // unconditionally, only valid lanes store
  const int sx = active ? s : P - 1;
  const int lo = UNI ? sx * SL : sx * K.yL + (sx < K.yr ? sx : K.yr);
  const int len = UNI ? SL : K.yL + (sx < K.yr ? 1 : 0);
  const int m = len - 1;  // interior rows (at least 2); row lo+m is the separator
  const bool z0 = (q == 0) && lo == 0;  // the (0,0) mode's first row: identity, right side 0
  const int pl = pq < g.nxh ? pq : g.nxh - 1;
  const double lam = K.lamx[pl] + K.lamz[kq];
  const C* __restrict__ Xl = K.spec + (int64_t)kq * K.ldx + pl;
  double xr[SL], xi[SL], ah[SL - 1], ch[SL - 1];
#pragma unroll
  for (int e = 0; e < SL; ++e) {
    const int row = (UNI || lo + e < g.ny) ? lo + e : g.ny - 1;
    const C v = Xl[(int64_t)row * nm];
    xr[e] = (double)v.x;
    xi[e] = (double)v.y;
  }
  if (K.zero_in && bid.x == 0) {
    // The (0,0) mode is the Neumann problem's singular one: its right-hand
    // side must have zero volume-weighted sum (compatibility), which the FP32
    // rounding of the forward transforms breaks; the gauge row phi_0 = 0
    // would then take the whole excess, at the wall, where 1/dy amplifies
    // it.  Removing the mean first leaves a uniform residual of the rounding's
    // size instead (and changes nothing for a compatible right-hand side).
    double pr = 0.0, pi = 0.0;
    if (lb == 0 && active) {
#pragma unroll
      for (int e = 0; e < SL; ++e)
        if (UNI || e < len) {
          pr += g.dy[lo + e] * xr[e];
          pi += g.dy[lo + e] * xi[e];
        }
    }
    if (lb == 0 && active) {
      A(0, s, 0) = pr;
      A(1, s, 0) = pi;
    }
    __syncthreads();
    if (lb == 0) {
      double Mr = 0.0, Mi = 0.0;
      for (int t = 0; t < P; ++t) {
        Mr += A(0, t, 0);
        Mi += A(1, t, 0);
      }
      Mr *= K.inv_sum_dy;
      Mi *= K.inv_sum_dy;
#pragma unroll
      for (int e = 0; e < SL; ++e) {
        xr[e] -= Mr;
        xi[e] -= Mi;
      }
    }
    __syncthreads();
  }
  double zr = xr[SL - 1], zi = xi[SL - 1];
  if (!UNI) {
#pragma unroll
    for (int e = 0; e < SL - 1; ++e)
      if (e == m) {
        zr = xr[e];
        zi = xi[e];
      }
  }
  // forward elimination of the interior rows: row e becomes
  //   x_e + ct_e x_{e+1} = dt_e - at_e z_left
  // in excess form (see excess_row): with u = 1 + ct and tau = 1 + at + ct
  // carried, every pivot and excess is a sum of terms of one sign
  double atp = -1.0, up = 1.0, tp = 0.0, dr = 0.0, di = 0.0;
  double tau[SL - 1];
#pragma unroll
  for (int e = 0; e < SL - 1; ++e)
    if (UNI || e < m) {
      const int j = lo + e;
      const bool idr = (e == 0 && z0);  // the gauge row: identity, right side 0
      const double a = idr ? 0.0 : K.ylo[j], c = idr ? 0.0 : K.yhi[j];
      const double inv = idr ? 1.0 : recip(lam - c - a * up);
      atp = -a * atp * inv;
      up = idr ? 1.0 : (lam - a * up) * inv;
      tp = idr ? 1.0 : (lam - a * tp) * inv;
      dr = idr ? 0.0 : (xr[e] - a * dr) * inv;
      di = idr ? 0.0 : (xi[e] - a * di) * inv;
      ah[e] = atp;
      ch[e] = c * inv;
      tau[e] = tp;
      xr[e] = dr;
      xi[e] = di;
    }
  // backward: x_e = d_e - ah_e z_left - ch_e z_right, with the excess
  // sg_e = 1 + ah_e + ch_e
  double ahl = 0.0, dlr = 0.0, dli = 0.0, sgl = 0.0, sg = 0.0;  // row m-1; sg: row e
#pragma unroll
  for (int e = SL - 2; e >= 0; --e)
    if (UNI || e < m) {
      if (e == m - 1) {
        ahl = ah[e];
        dlr = xr[e];
        dli = xi[e];
        sgl = tau[e];
        sg = sgl;
      } else {
        const double ct = ch[e];
        xr[e] -= ct * xr[e + 1];
        xi[e] -= ct * xi[e + 1];
        ah[e] -= ct * ah[e + 1];
        ch[e] = -ct * ch[e + 1];
        sg = tau[e] - ct * sg;
      }
    }
  // the first interior row of each segment, for the separator row before it
  // (its excess in slot 9, free until the separators are solved)
  if (active) {
    A(1, s, lb) = ch[0];
    A(2, s, lb) = xr[0];
    A(3, s, lb) = xi[0];
    A(9, s, lb) = sg;
  }
  __syncthreads();
  if (active) {
    const int jz = lo + m;
    const double az = K.ylo[jz], cz = K.yhi[jz];
    double rg = 0.0, rdr = zr - az * dlr, rdi = zi - az * dli;
    double re = lam - az * sgl - cz;
    if (s + 1 < P) {
      re = lam - az * sgl - cz * A(9, s + 1, lb);
      rg = -cz * A(1, s + 1, lb);
      rdr -= cz * A(2, s + 1, lb);
      rdi -= cz * A(3, s + 1, lb);
    }
    A(4, s, lb) = -az * ahl;
    A(5, s, lb) = re;
    A(6, s, lb) = rg;
    A(7, s, lb) = rdr;
    A(8, s, lb) = rdi;
  }
  __syncthreads();
  {
    // transposed: lane (mode lt, separator st), PP lanes per mode; rows past
    // P act as identity rows (excess 1).  Each step eliminates the
    // neighbours at distance `step`; a neighbour outside 0..PP-1 is an
    // identity row, which contributes nothing (its multiplier is 0), so the
    // lane reads itself there and drops the term.
    const int lt = threadIdx.x / PP, st = threadIdx.x % PP;
    const int grp = (threadIdx.x & 63) - st;
    const bool own = lt < TL && st < P;
    double ra = 0.0, re = 1.0, rg = 0.0, rdr = 0.0, rdi = 0.0;
    if (own) {
      ra = A(4, st, lt);
      re = A(5, st, lt);
      rg = A(6, st, lt);
      rdr = A(7, st, lt);
      rdi = A(8, st, lt);
    }
    for (int step = 1; step < PP; step <<= 1) {
      const int im = st - step, ip = st + step;
      const bool hm = im >= 0, hp = ip < PP;
      const int sm_ = grp + (hm ? im : st), sp_ = grp + (hp ? ip : st);
      const double rib = recip(re - ra - rg);  // neighbours divide by this row's pivot
      const double am = lane_read(ra, sm_), rm = lane_read(rib, sm_), em = lane_read(re, sm_);
      const double dmr = lane_read(rdr, sm_), dmi = lane_read(rdi, sm_);
      const double gp = lane_read(rg, sp_), rp = lane_read(rib, sp_), ep = lane_read(re, sp_);
      const double dpr = lane_read(rdr, sp_), dpi = lane_read(rdi, sp_);
      const double k1 = hm ? ra * rm : 0.0, k2 = hp ? rg * rp : 0.0;
      excess_row(ra, re, rg, k1, am, em, k2, gp, ep);
      rdr = rdr - dmr * k1 - dpr * k2;
      rdi = rdi - dmi * k1 - dpi * k2;
    }
    if (own) {
      const double rib = recip(re - ra - rg);
      A(9, st, lt) = rdr * rib;
      A(10, st, lt) = rdi * rib;
    }
  }
  __syncthreads();
  const double zRr = A(9, s, lb), zRi = A(10, s, lb);
  const double zLr = (s > 0) ? A(9, s - 1, lb) : 0.0;
  const double zLi = (s > 0) ? A(10, s - 1, lb) : 0.0;
#pragma unroll
  for (int e = 0; e < SL - 1; ++e)
    if (UNI || e < m) {
      xr[e] = xr[e] - ah[e] * zLr - ch[e] * zRr;
      xi[e] = xi[e] - ah[e] * zLi - ch[e] * zRi;
    }
  zr = zRr;
  zi = zRi;
  if (bid.x == 0) {
    // zero volume-weighted mean of the (0,0) mode (lane 0 of block 0):
    // per-segment partial sums, then their sum in segment order
    double pr = 0.0, pi = 0.0;
    if (lb == 0) {
#pragma unroll
      for (int e = 0; e < SL; ++e)
        if (UNI || e < len) {
          const double dyj = g.dy[lo + e];
          pr += dyj * (e < m ? xr[e] : zr);
          pi += dyj * (e < m ? xi[e] : zi);
        }
    }
    __syncthreads();
    if (lb == 0) {
      A(0, s, 0) = pr;
      A(1, s, 0) = pi;
    }
    __syncthreads();
    if (lb == 0) {
      double Mr = 0.0, Mi = 0.0;
      for (int t = 0; t < P; ++t) {
        Mr += A(0, t, 0);
        Mi += A(1, t, 0);
      }
      Mr *= K.inv_sum_dy;
      Mi *= K.inv_sum_dy;
#pragma unroll
      for (int e = 0; e < SL - 1; ++e)
        if (UNI || e < m) {
          xr[e] -= Mr;
          xi[e] -= Mi;
        }
      zr -= Mr;
      zi -= Mi;
    }
  }
  if (valid) {
    // an FP32 spectrum hands the (0,0) mode (a real column) to the inverse x
    // pass in FP64, so that the zero-mean gauge survives the FP32 rounding
    const bool keep = (q == 0) && K.zm;
    const int64_t nmo = (int64_t)g.nz * K.ldx_out;
    CO* __restrict__ X = (K.spec_out ? static_cast<CO*>(K.spec_out) : reinterpret_cast<CO*>(K.spec)) +
                         (int64_t)kq * K.ldx_out + pq;
#pragma unroll
    for (int e = 0; e < SL; ++e)
      if (UNI || e < len) {
        const double vr = (e < m) ? xr[e] : zr;
        const double vi = (e < m) ? xi[e] : zi;
        if (keep) K.zm[lo + e] = vr;
        X[(int64_t)(lo + e) * nmo] = keep ? mkc<CO>((RO)0, (RO)0) : mkc<CO>((RO)vr, (RO)vi);
      }
  }
}

// The same solve with the separator system reduced block-wide in LDS, for
// modes of more than 64 separators (P rounded up past one wavefront).
template <typename C, typename CO, bool G = false>
__global__ __launch_bounds__(1024) void k_tri_y_blk(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using RO = typename RealOf<CO>::T;
  if (gated(K)) return;
  extern __shared__ __align__(16) unsigned char smraw[];
  double* sm = reinterpret_cast<double*>(smraw);  // 7 arrays of P doubles per line
  const GridView& g = K.g;
  const int TL = K.ytl, P = K.yP;
  const int lb = threadIdx.x % TL, s = threadIdx.x / TL;
  // modes q = k ldx + p over the padded rows; padding columns are skipped
  const int64_t nm = (int64_t)g.nz * K.ldx;
  const int64_t q = (int64_t)bid.x * TL + lb;
  const bool valid = q < nm && (int)(q % K.ldx) < g.nxh;
  auto at = [&](int f, int seg) -> double& { return sm[((size_t)f * P + seg) * TL + lb]; };
  const int lo = s * K.yL + (s < K.yr ? s : K.yr);
  const int len = K.yL + (s < K.yr ? 1 : 0);
  const int m = len - 1;  // interior rows (at least 2); row lo+m is the separator
  const bool zero = (q == 0);
  // lanes past the last mode solve a harmless non-singular system
  const double lam = valid ? K.lamx[q % K.ldx] + K.lamz[q / K.ldx] : -1.0;
  C* __restrict__ X = K.spec + q;
  double xr[YL], xi[YL], ah[YL], ch[YL];
  double zr = 0.0, zi = 0.0;
#pragma unroll
  for (int e = 0; e < YL; ++e) {
    xr[e] = 0.0;
    xi[e] = 0.0;
    ah[e] = 0.0;
    ch[e] = 0.0;
  }
  if (valid) {
#pragma unroll
    for (int e = 0; e < YL; ++e)
      if (e < len) {
        const C v = X[(int64_t)(lo + e) * nm];
        if (e < m) {
          xr[e] = (double)v.x;
          xi[e] = (double)v.y;
        } else {
          zr = (double)v.x;
          zi = (double)v.y;
        }
      }
  }
  if (K.zero_in && bid.x == 0) {
    // the (0,0) mode's right-hand side loses its volume-weighted mean (see
    // the wavefront form of this solve)
    double pr = 0.0, pi = 0.0;
    if (lb == 0) {
#pragma unroll
      for (int e = 0; e < YL; ++e)
        if (e < len) {
          const double dyj = g.dy[lo + e];
          pr += dyj * (e < m ? xr[e] : zr);
          pi += dyj * (e < m ? xi[e] : zi);
        }
      at(0, s) = pr;
      at(1, s) = pi;
    }
    __syncthreads();
    if (lb == 0) {
      double Mr = 0.0, Mi = 0.0;
      for (int t = 0; t < P; ++t) {
        Mr += sm[((size_t)0 * P + t) * TL];
        Mi += sm[((size_t)1 * P + t) * TL];
      }
      Mr *= K.inv_sum_dy;
      Mi *= K.inv_sum_dy;
#pragma unroll
      for (int e = 0; e < YL; ++e) {
        xr[e] -= Mr;
        xi[e] -= Mi;
      }
      zr -= Mr;
      zi -= Mi;
    }
    __syncthreads();
  }
  // forward elimination of the interior rows: row e becomes
  //   x_e + ct_e x_{e+1} = dt_e - at_e z_left
  // in excess form (see excess_row and the wavefront form of this solve)
  double atp = -1.0, up = 1.0, tp = 0.0, dr = 0.0, di = 0.0;
  double tau[YL - 1];
#pragma unroll
  for (int e = 0; e < YL - 1; ++e)
    if (e < m) {
      const int j = lo + e;
      const bool idr = zero && j == 0;  // the gauge row: identity, right side 0
      const double a = idr ? 0.0 : K.ylo[j], c = idr ? 0.0 : K.yhi[j];
      const double inv = idr ? 1.0 : 1.0 / (lam - c - a * up);
      atp = -a * atp * inv;
      up = idr ? 1.0 : (lam - a * up) * inv;
      tp = idr ? 1.0 : (lam - a * tp) * inv;
      dr = idr ? 0.0 : (xr[e] - a * dr) * inv;
      di = idr ? 0.0 : (xi[e] - a * di) * inv;
      ah[e] = atp;
      ch[e] = c * inv;
      tau[e] = tp;
      xr[e] = dr;
      xi[e] = di;
    }
  // backward: x_e = d_e - ah_e z_left - ch_e z_right, excess 1 + ah_e + ch_e
  double ahl = 0.0, dlr = 0.0, dli = 0.0, sgl = 0.0, sg = 0.0;  // row m-1; sg: row e
#pragma unroll
  for (int e = YL - 2; e >= 0; --e)
    if (e < m) {
      if (e == m - 1) {
        ahl = ah[e];
        dlr = xr[e];
        dli = xi[e];
        sgl = tau[e];
        sg = sgl;
      } else {
        const double ct = ch[e];
        xr[e] -= ct * xr[e + 1];
        xi[e] -= ct * xi[e + 1];
        ah[e] -= ct * ah[e + 1];
        ch[e] = -ct * ch[e + 1];
        sg = tau[e] - ct * sg;
      }
    }
  // the first interior row of each segment, for the separator row before it
  at(0, s) = sg;
  at(1, s) = ch[0];
  at(2, s) = xr[0];
  at(3, s) = xi[0];
  __syncthreads();
  const int jz = lo + m;
  const double az = K.ylo[jz], cz = K.yhi[jz];
  double ra = -az * ahl, re = lam - az * sgl - cz, rg = 0.0;
  double rdr = zr - az * dlr, rdi = zi - az * dli;
  if (s + 1 < P) {
    re = lam - az * sgl - cz * at(0, s + 1);
    rg = -cz * at(1, s + 1);
    rdr -= cz * at(2, s + 1);
    rdi -= cz * at(3, s + 1);
  }
  __syncthreads();
  at(0, s) = ra;
  at(1, s) = re;
  at(2, s) = rg;
  at(3, s) = rdr;
  at(4, s) = rdi;
  __syncthreads();
  // parallel cyclic reduction in excess form; rows outside 0..P-1 act as
  // identity rows (multiplier 0)
  for (int st = 1; st < P; st <<= 1) {
    const int im = s - st, ip = s + st;
    double am = 0.0, em = 1.0, dmr = 0.0, dmi = 0.0, k1 = 0.0;
    double gp = 0.0, ep = 1.0, dpr = 0.0, dpi = 0.0, k2 = 0.0;
    if (im >= 0) {
      am = at(0, im);
      em = at(1, im);
      dmr = at(3, im);
      dmi = at(4, im);
      k1 = ra / (em - am - at(2, im));
    }
    if (ip < P) {
      gp = at(2, ip);
      ep = at(1, ip);
      dpr = at(3, ip);
      dpi = at(4, ip);
      k2 = rg / (ep - at(0, ip) - gp);
    }
    double na = ra, ne = re, ng = rg;
    excess_row(na, ne, ng, k1, am, em, k2, gp, ep);
    const double ndr = rdr - dmr * k1 - dpr * k2;
    const double ndi = rdi - dmi * k1 - dpi * k2;
    __syncthreads();
    ra = na;
    re = ne;
    rg = ng;
    rdr = ndr;
    rdi = ndi;
    at(0, s) = ra;
    at(1, s) = re;
    at(2, s) = rg;
    at(3, s) = rdr;
    at(4, s) = rdi;
    __syncthreads();
  }
  const double rb = re - ra - rg;
  at(5, s) = rdr / rb;
  at(6, s) = rdi / rb;
  __syncthreads();
  const double zRr = at(5, s), zRi = at(6, s);
  const double zLr = (s > 0) ? at(5, s - 1) : 0.0;
  const double zLi = (s > 0) ? at(6, s - 1) : 0.0;
#pragma unroll
  for (int e = 0; e < YL - 1; ++e)
    if (e < m) {
      xr[e] = xr[e] - ah[e] * zLr - ch[e] * zRr;
      xi[e] = xi[e] - ah[e] * zLi - ch[e] * zRi;
    }
  zr = zRr;
  zi = zRi;
  if (bid.x == 0) {
    // zero volume-weighted mean of the (0,0) mode (lane 0 of block 0):
    // per-segment partial sums, then their sum in segment order
    double pr = 0.0, pi = 0.0;
    if (lb == 0) {
#pragma unroll
      for (int e = 0; e < YL; ++e)
        if (e < len) {
          const double dyj = g.dy[lo + e];
          pr += dyj * (e < m ? xr[e] : zr);
          pi += dyj * (e < m ? xi[e] : zi);
        }
    }
    __syncthreads();
    if (lb == 0) {
      at(0, s) = pr;
      at(1, s) = pi;
    }
    __syncthreads();
    if (lb == 0) {
      double Mr = 0.0, Mi = 0.0;
      for (int t = 0; t < P; ++t) {
        Mr += at(0, t);
        Mi += at(1, t);
      }
      Mr *= K.inv_sum_dy;
      Mi *= K.inv_sum_dy;
#pragma unroll
      for (int e = 0; e < YL - 1; ++e)
        if (e < m) {
          xr[e] -= Mr;
          xi[e] -= Mi;
        }
      zr -= Mr;
      zi -= Mi;
    }
  }
  if (valid) {
    // an FP32 spectrum hands the (0,0) mode (a real column) to the inverse x
    // pass in FP64, so that the zero-mean gauge survives the FP32 rounding
    const bool keep = zero && K.zm;
    const int64_t nmo = (int64_t)g.nz * K.ldx_out;
    CO* __restrict__ XO = (K.spec_out ? static_cast<CO*>(K.spec_out) : reinterpret_cast<CO*>(K.spec)) +
                          (q / K.ldx) * K.ldx_out + q % K.ldx;
#pragma unroll
    for (int e = 0; e < YL; ++e)
      if (e < len) {
        const double vr = (e < m) ? xr[e] : zr;
        const double vi = (e < m) ? xi[e] : zi;
        if (keep) K.zm[lo + e] = vr;
        XO[(int64_t)(lo + e) * nmo] = keep ? mkc<CO>((RO)0, (RO)0) : mkc<CO>((RO)vr, (RO)vi);
      }
  }
}

template <typename C, bool G = false>
__global__ __launch_bounds__(256) void k_fftx_inv(GArg<PoisK<C>, G> grp_arg_) {
  uint3 bid, gdim;
  const PoisK<C>& K = grp_enter<PoisK<C>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using R = typename RealOf<C>::T;
  if (gated(K)) return;
  extern __shared__ __align__(16) unsigned char smraw[];
  C* sm = reinterpret_cast<C*>(smraw);
  const GridView& g = K.g;
  const int nx = g.nx, nxh = g.nxh;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int64_t row0 = (int64_t)bid.x * K.rows;
  const int nr = (int)((row0 + K.rows <= nrows) ? K.rows : nrows - row0);
  // two half spectra per complex sequence: Z = A + iB over the Hermitian
  // extension (the bins 0 and nx/2 of a real sequence are real), so that the
  // real and imaginary parts of the inverse are rows 2c and 2c+1
  auto bin = [&](int r, int k) -> C {
    if (r >= nr) return mkc<C>((R)0, (R)0);
    C c = (k < nxh) ? K.spec[(row0 + r) * K.ldx + k] : K.spec[(row0 + r) * K.ldx + (nx - k)];
    if (k >= nxh) c.y = -c.y;
    if (k == 0 || 2 * k == nx) c.y = (R)0;
    return c;
  };
  for (int e = threadIdx.x; e < (K.rows / 2) * nx; e += blockDim.x) {
    const int col = e / nx, k = e % nx;
    const C A = bin(2 * col, k), B = bin(2 * col + 1, k);
    sm[e] = mkc<C>(A.x - B.y, A.y + B.x);
  }
  __syncthreads();
  const C* out = lds_fft<C, true>(sm, sm + (K.rows / 2) * nx, K.px, K.rows / 2, 1, nx);
  const R* sr = reinterpret_cast<const R*>(out);
  for (int e = threadIdx.x; e < nr * nx; e += blockDim.x) {
    const int r = e / nx, i = e % nx;
    double v = (double)sr[2 * ((r >> 1) * nx + i) + (r & 1)] * K.scale;
    if (K.zm) v += K.zm[(int)((row0 + e / nx) / g.nz)] * K.scale;
    if (K.msum) v -= *K.msum * K.inv_vtot;
    if (K.accumulate)
      K.phi[row0 * nx + e] += v;
    else
      K.phi[row0 * nx + e] = v;
  }
}

// Sum of the per-block partials of phi dV in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int n,
                                                      double* __restrict__ out, const u64* gate,
                                                      double gate_tol) {
  if (gate && __longlong_as_double((long long)*gate) <= gate_tol) return;
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// Refinement bookkeeping after one mixed solve: rmax[k] (k = 1..nref) is the
// residual that opened refinement k (0 if it never ran), rmax[nref+1] the
// final check.  stats: [solves, corrections, largest final max|r| * adt,
// largest max|r| * adt after the first correction, largest max|r| * adt of
// the initial solve, sum over solves of that initial value].
__global__ void k_refine_stats(const u64* rmax, int nref, double tol, double adt, double* stats,
                               uint32_t* flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int k = 1, corr = 0;
  double last = __longlong_as_double((long long)rmax[1]);
  while (k <= nref && !(last <= tol)) {
    ++corr;
    ++k;
    last = __longlong_as_double((long long)rmax[k]);
  }
  if (!(last <= tol)) atomicOr(flags, last == last ? FLAG_REFINE : FLAG_NONFINITE);
  stats[0] += 1.0;
  stats[1] += (double)corr;
  const double fin = last * adt;
  if (!(fin <= stats[2])) stats[2] = fin;
  // the residual left by the first correction (0 when none was needed)
  const double r2 = (nref >= 2) ? __longlong_as_double((long long)rmax[2]) * adt : 0.0;
  if (!(r2 <= stats[3])) stats[3] = r2;
  const double r1 = __longlong_as_double((long long)rmax[1]) * adt;
  if (!(r1 <= stats[4])) stats[4] = r1;
  stats[5] += r1;
}

template <typename C>
static PlanDev<C> to_dev(const FFTPlan* p, const C* tw) {
  PlanDev<C> d;
  d.n = p->n;
  d.nst = p->nst;
  for (int i = 0; i < 16; ++i) d.radix[i] = p->radix[i];
  d.tw = tw;
  return d;
}

// x-rows per block and x-modes per z-pass block for a spectrum type
template <typename C>
static void pass_shape(const GridView& g, PoisK<C>& K) {
  // per block two LDS buffers of at most fft_buf complex values: x passes
  // take an even number of real rows, two per complex sequence (nx and nz
  // <= fft_buf, checked when the context is created)
  int rows = 2 * (fft_buf<C>() / g.nx);
  if (rows > 32) rows = 32;
  K.rows = rows;
  int tp = fft_buf<C>() / g.nz;
  if (tp > 16) tp = 16;
  K.tp = tp;
}

// The five passes of a solve.  K (spectrum type C) runs the forward x and z
// passes and the wall-normal solve; KI (type CI) the inverse z and x passes.
// With CI != C the solve writes KI's spectrum (its own precision and row
// stride): the refined mixed form transforms forward in FP32 and back in
// FP64.
template <typename C, typename CI>
static void run_passes(Prof* pf, hipStream_t s, const GridView& g, PoisK<C> K, PoisK<CI> KI) {
  constexpr int CB = (int)sizeof(C), CBI = (int)sizeof(CI);
  pass_shape<C>(g, K);
  pass_shape<CI>(g, KI);
  const int rows = K.rows, tp = K.tp;
  line_plan(g.ny, false, YL, &K.yP, &K.yL, &K.yr);
  // more than 64 separators of 6-row segments: 12-row segments when that
  // brings a mode's separators into one wavefront
  int sl = YL;
  if (K.yP > 64) {
    int P2, L2, r2;
    line_plan(g.ny, false, 2 * YL, &P2, &L2, &r2);
    if (P2 <= 64) {
      sl = 2 * YL;
      K.yP = P2;
      K.yL = L2;
      K.yr = r2;
    }
  }
  K.yPP = 1;
  while (K.yPP < K.yP) K.yPP <<= 1;
  // separators of one mode in one wavefront when they fit; else block-wide.
  // Wavefront form: 8 modes per block once a mode has 32 or more separators
  // (blocks of 256-512 threads: more blocks per CU; 128-byte row pieces)
  const bool ywave = K.yPP <= 64;
  K.ytl = ywave ? (K.yPP >= 32 ? 8 : 1024 / K.yPP) : 1024 / K.yP;
  if (K.ytl > 16) K.ytl = 16;
  if (K.ytl < 1) K.ytl = 1;
  const int64_t nrows = (int64_t)g.ny * g.nz;
  const int xblocks = (int)((nrows + rows - 1) / rows);
  const int xblocks_i = (int)((nrows + KI.rows - 1) / KI.rows);
  const size_t xsh = 2 * (size_t)(rows / 2) * g.nx * CB;
  const size_t xsh_i = 2 * (size_t)(KI.rows / 2) * g.nx * CBI;
  const size_t zsh = 2 * (size_t)tp * g.nz * CB;
  const size_t zsh_i = 2 * (size_t)KI.tp * g.nz * CBI;
  const dim3 zgrid((g.nxh + tp - 1) / tp, g.ny), zgrid_i((g.nxh + KI.tp - 1) / KI.tp, g.ny);
  K.ldx = spec_ld(g.nxh, sizeof(C) == sizeof(float2));
  KI.ldx = spec_ld(g.nxh, sizeof(CI) == sizeof(float2));
  const bool split = (void*)KI.spec != (void*)K.spec;
  K.spec_out = split ? (void*)KI.spec : nullptr;
  K.ldx_out = split ? KI.ldx : K.ldx;
  K.zero_in = split ? 1 : 0;
  const int64_t nm = (int64_t)g.nz * K.ldx;
  const int yblocks = (int)((nm + K.ytl - 1) / K.ytl);
  // wavefront form: z-major blocks of ytl modes of one z row
  const int ywblocks = g.nz * ((g.nxh + K.ytl - 1) / K.ytl);
  const size_t ysh = ywave ? 11 * sizeof(double) * (size_t)K.yPP * (K.ytl + 1)
                           : 7 * sizeof(double) * (size_t)K.yP * K.ytl;
  const bool resid = K.mode >= SRC_RESIDUAL;
  // length-256 x transforms: 2 X16_SC rows per block
  const bool x256 = (g.nx == 256 && K.ldx <= X16_LDX_MAX);
  const bool x256_i = (g.nx == 256 && KI.ldx <= X16_LDX_MAX);
  const int xb = x256 ? (int)((nrows + 2 * X16_SC - 1) / (2 * X16_SC)) : xblocks;
  const int xb_i = x256_i ? (int)((nrows + 2 * X16_SC - 1) / (2 * X16_SC)) : xblocks_i;
  if (x256)
    IBM_LAUNCH_G(pf, resid ? "pois_resid_fftx" : "pois_fftx_fwd", s, (&k_fftx256_fwd<C, true>), dim3(xb), dim3(32 * X16_SC), 0, K, k_fftx256_fwd<C><<<xb, 32 * X16_SC, 0, s>>>(K));
  else
    IBM_LAUNCH_G(pf, resid ? "pois_resid_fftx" : "pois_fftx_fwd", s, (&k_fftx_fwd<C, true>), dim3(xblocks), dim3(256), xsh, K, k_fftx_fwd<C><<<xblocks, 256, xsh, s>>>(K));
  if (K.mode == SRC_CHECK) return;
  if (resid) {
    K.gate = K.rmax;  // the rest of a refinement runs only if its residual is too large
    KI.gate = K.rmax;
    KI.gate_tol = K.gate_tol;
    IBM_LAUNCH(pf, "pois_mean", s,
               (k_sum_partials<<<1, 256, 0, s>>>(K.psum, xb, const_cast<double*>(K.msum),
                                                  K.gate, K.gate_tol)));
  }
  const bool z256 = (g.nz == 256);
  const dim3 z16grid((g.nxh + Z16_TC - 1) / Z16_TC, g.ny);
  // lengths 512 and 1024: 8 and 4 modes per block, XCD-aware 1-D grids
  const unsigned z512b = (unsigned)zline_blocks(zline_group<C, 8>(), (g.nxh + 7) / 8, g.ny);
  const unsigned z1kb = (unsigned)zline_blocks(zline_group<C, 4>(), (g.nxh + 3) / 4, g.ny);
  const unsigned z512b_i = (unsigned)zline_blocks(zline_group<CI, 8>(), (g.nxh + 7) / 8, g.ny);
  const unsigned z1kb_i = (unsigned)zline_blocks(zline_group<CI, 4>(), (g.nxh + 3) / 4, g.ny);
  if (z256)
    IBM_LAUNCH_G(pf, "pois_fftz_fwd", s, (&k_fftz256<C, false, true>), dim3(z16grid), dim3(16 * Z16_TC), 0, K, k_fftz256<C, false><<<z16grid, 16 * Z16_TC, 0, s>>>(K));
  else if (g.nz == 512)
    IBM_LAUNCH_G(pf, "pois_fftz_fwd", s, (&k_fftz4s<C, false, 2, true>), dim3(z512b), dim3(256), 0, K, k_fftz4s<C, false, 2><<<z512b, 256, 0, s>>>(K));
  else if (g.nz == 1024)
    IBM_LAUNCH_G(pf, "pois_fftz_fwd", s, (&k_fftz4s<C, false, 4, true>), dim3(z1kb), dim3(256), 0, K, k_fftz4s<C, false, 4><<<z1kb, 256, 0, s>>>(K));
  else
    IBM_LAUNCH_G(pf, "pois_fftz_fwd", s, (&k_fftz<C, false, true>), dim3(zgrid), dim3(256), zsh, K, k_fftz<C, false><<<zgrid, 256, zsh, s>>>(K));
  if (ywave && sl == 2 * YL && K.yr == 0 && K.yL == sl)
    IBM_LAUNCH_G(pf, "pois_tri_y", s, (&k_tri_y<C, true, CI, 2 * YL, true>), dim3(ywblocks), dim3(K.ytl * K.yPP), ysh, K, k_tri_y<C, true, CI, 2 * YL><<<ywblocks, K.ytl * K.yPP, ysh, s>>>(K));
  else if (ywave && sl == 2 * YL)
    IBM_LAUNCH_G(pf, "pois_tri_y", s, (&k_tri_y<C, false, CI, 2 * YL, true>), dim3(ywblocks), dim3(K.ytl * K.yPP), ysh, K, k_tri_y<C, false, CI, 2 * YL><<<ywblocks, K.ytl * K.yPP, ysh, s>>>(K));
  else if (ywave && K.yr == 0 && K.yL == YL)
    IBM_LAUNCH_G(pf, "pois_tri_y", s, (&k_tri_y<C, true, CI, YL, true>), dim3(ywblocks), dim3(K.ytl * K.yPP), ysh, K, k_tri_y<C, true, CI, YL><<<ywblocks, K.ytl * K.yPP, ysh, s>>>(K));
  else if (ywave)
    IBM_LAUNCH_G(pf, "pois_tri_y", s, (&k_tri_y<C, false, CI, YL, true>), dim3(ywblocks), dim3(K.ytl * K.yPP), ysh, K, k_tri_y<C, false, CI, YL><<<ywblocks, K.ytl * K.yPP, ysh, s>>>(K));
  else
    IBM_LAUNCH_G(pf, "pois_tri_y", s, (&k_tri_y_blk<C, CI, true>), dim3(yblocks), dim3(K.ytl * K.yP), ysh, K, k_tri_y_blk<C, CI><<<yblocks, K.ytl * K.yP, ysh, s>>>(K));
  if (z256)
    IBM_LAUNCH_G(pf, "pois_fftz_inv", s, (&k_fftz256<CI, true, true>), dim3(z16grid), dim3(16 * Z16_TC), 0, KI, k_fftz256<CI, true><<<z16grid, 16 * Z16_TC, 0, s>>>(KI));
  else if (g.nz == 512)
    IBM_LAUNCH_G(pf, "pois_fftz_inv", s, (&k_fftz4s<CI, true, 2, true>), dim3(z512b_i), dim3(256), 0, KI, k_fftz4s<CI, true, 2><<<z512b_i, 256, 0, s>>>(KI));
  else if (g.nz == 1024)
    IBM_LAUNCH_G(pf, "pois_fftz_inv", s, (&k_fftz4s<CI, true, 4, true>), dim3(z1kb_i), dim3(256), 0, KI, k_fftz4s<CI, true, 4><<<z1kb_i, 256, 0, s>>>(KI));
  else
    IBM_LAUNCH_G(pf, "pois_fftz_inv", s, (&k_fftz<CI, true, true>), dim3(zgrid_i), dim3(256), zsh_i, KI, k_fftz<CI, true><<<zgrid_i, 256, zsh_i, s>>>(KI));
  // lengths 512 and 1024: one sequence (two rows) per 32 or 64 lanes, 2 x
  // 4096/nx rows per block of 256 threads
  const int rpb4 = (g.nx == 512 || g.nx == 1024) ? 2 * (4096 / g.nx) : 1;
  const int xb4_i = (int)((nrows + rpb4 - 1) / rpb4);
  if (x256_i)
    IBM_LAUNCH_G(pf, "pois_fftx_inv", s, (&k_fftx256_inv<CI, true>), dim3(xb_i), dim3(32 * X16_SC), 0, KI, k_fftx256_inv<CI><<<xb_i, 32 * X16_SC, 0, s>>>(KI));
  else if (g.nx == 1024)
    IBM_LAUNCH_G(pf, "pois_fftx_inv", s, (&k_fftx4s_inv<CI, 4, true>), dim3(xb4_i), dim3(256), 0, KI, k_fftx4s_inv<CI, 4><<<xb4_i, 256, 0, s>>>(KI));
  else if (g.nx == 512)
    IBM_LAUNCH_G(pf, "pois_fftx_inv", s, (&k_fftx4s_inv<CI, 2, true>), dim3(xb4_i), dim3(256), 0, KI, k_fftx4s_inv<CI, 2><<<xb4_i, 256, 0, s>>>(KI));
  else
    IBM_LAUNCH_G(pf, "pois_fftx_inv", s, (&k_fftx_inv<CI, true>), dim3(xblocks_i), dim3(256), xsh_i, KI, k_fftx_inv<CI><<<xblocks_i, 256, xsh_i, s>>>(KI));
}

// the inverse passes' view of a solve: the fields the inverse z and x
// passes read, over the spectrum `spec` of type CI
template <typename CI, typename C>
static PoisK<CI> inverse_view(const PoisK<C>& K, const PoissonArgs& a, void* spec) {
  PoisK<CI> I{};
  I.g = K.g;
  const bool f32 = sizeof(CI) == sizeof(float2);
  I.px = to_dev<CI>(a.px, reinterpret_cast<const CI*>(f32 ? (const void*)a.px->tw32
                                                           : (const void*)a.px->tw));
  I.pz = to_dev<CI>(a.pz, reinterpret_cast<const CI*>(f32 ? (const void*)a.pz->tw32
                                                           : (const void*)a.pz->tw));
  I.mode = K.mode;
  I.spec = static_cast<CI*>(spec);
  I.phi = K.phi;
  I.accumulate = K.accumulate;
  I.scale = K.scale;
  I.msum = K.msum;
  I.inv_vtot = K.inv_vtot;
  I.zm = K.zm;
  I.gate = K.gate;
  I.gate_tol = K.gate_tol;
  return I;
}

// one run of the five passes: FP64 throughout, or (refined mixed form) the
// forward passes on the FP32 spectrum and the inverse ones on the FP64
// spectrum a.spec64
template <typename C>
static void passes(Prof* pf, hipStream_t s, const GridView& g, const PoissonArgs& a,
                   const PoisK<C>& K) {
  if constexpr (sizeof(C) == sizeof(float2)) {
    if (a.spec64) {
      run_passes<C, double2>(pf, s, g, K, inverse_view<double2>(K, a, a.spec64));
      return;
    }
  }
  run_passes<C, C>(pf, s, g, K, K);
}

template <typename C>
static void solve(Prof* pf, hipStream_t s, const GridView& g, const PoissonArgs& a,
                  const C* twx, const C* twz, const double* rhs, const double* u,
                  const double* v, const double* w, const uint32_t* cb_mask, const double* qf,
                  const void* p, double inv_adt, double* phi) {
  PoisK<C> K{};
  K.g = g;
  K.px = to_dev<C>(a.px, twx);
  K.pz = to_dev<C>(a.pz, twz);
  K.mode = rhs ? SRC_ARRAY : SRC_VELOCITY;
  K.rhs = rhs;
  K.u = u;
  K.v = v;
  K.w = w;
  K.cb_mask = cb_mask;
  K.qf = qf;
  K.pq = p;
  K.pq32 = a.p_fp32;
  K.inv_adt = inv_adt;
  K.spec = reinterpret_cast<C*>(a.spec);
  K.lamx = a.lamx;
  K.lamz = a.lamz;
  K.ylo = a.ylo;
  K.yhi = a.yhi;
  K.inv_sum_dy = 1.0 / a.sum_dy;
  K.scale = 1.0 / ((double)g.nx * g.nz);
  K.phi = phi;
  const int nref = a.refine ? a.nref : 0;
  K.rhs_keep = a.refine ? a.rhs_keep : nullptr;
  // with an FP64 spectrum after the wall-normal solve the (0,0) mode needs
  // no FP64 side column
  K.zm = (a.fp32 && !a.spec64) ? a.zm : nullptr;
  // the tolerance bounds max|r| * alpha dt
  K.gate_tol = a.tol * inv_adt;
  if (a.refine) launch_fill_u64(pf, s, a.rmax, nref + 2, 0ull);
  passes<C>(pf, s, g, a, K);
  if (!a.refine) return;
  K.rhs = a.rhs_keep;
  K.rhs_keep = nullptr;
  K.phi_in = phi;
  K.accumulate = 1;
  K.inv_vtot = 1.0 / a.vtot;
  for (int k = 1; k <= nref + 1; ++k) {
    K.mode = (k <= nref) ? SRC_RESIDUAL : SRC_CHECK;
    K.rmax = a.rmax + k;
    K.gate = (k > 1) ? a.rmax + (k - 1) : nullptr;
    K.psum = (k <= nref) ? a.psum : nullptr;
    K.msum = (k <= nref) ? a.msum + k : nullptr;
    passes<C>(pf, s, g, a, K);
  }
  IBM_LAUNCH(pf, "pois_refine_stats", s,
             (k_refine_stats<<<1, 64, 0, s>>>(a.rmax, nref, K.gate_tol, 1.0 / inv_adt, a.stats,
                                              a.flags)));
}

void launch_poisson(Prof* pf, hipStream_t s, const GridView& g, const PoissonArgs& a,
                    const double* rhs, const double* u, const double* v, const double* w,
                    const uint32_t* cb_mask, const double* qf, const void* p, double inv_adt,
                    double* phi) {
  if (a.fp32)
    solve<float2>(pf, s, g, a, a.px->tw32, a.pz->tw32, rhs, u, v, w, cb_mask, qf, p, inv_adt,
                  phi);
  else
    solve<double2>(pf, s, g, a, a.px->tw, a.pz->tw, rhs, u, v, w, cb_mask, qf, p, inv_adt, phi);
}

}  // namespace ibm
