// Consistent mass correction (paper Sec. 3.2, Eqs. mod_div, q_boundary, q_F,
// elliptic_mod):
//   A   = sum over C_B of (D u_hat) dV,   V_B = sum over C_B of dV,
//   q_F = -A / |C_F|,  |C_F| = V_total - V_B,
//   rhs = (D u_hat - q_F)/(alpha dt) on C_F and 0 on C_B.
// The sums run over the sorted C_B list only (O(surface) work), in a fixed
// two-level order (a fixed partition into blocks, a fixed tree inside each
// block, then a fixed tree over the block partials), so the result is
// reproducible bit for bit from run to run.  No floating-point atomics.
#include "geom.h"

namespace ibm {

constexpr int MB = 256;   // blocks of the first level
constexpr int MT = 256;   // threads per block

__device__ __forceinline__ double div_at(const GridView& g, const double* u, const double* v,
                                         const double* w, int64_t cell) {
  const int64_t plane = (int64_t)g.nz * g.nx;
  const int i = (int)(cell % g.nx);
  const int k = (int)((cell / g.nx) % g.nz);
  const int j = (int)(cell / plane);
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const int64_t row = (int64_t)j * plane + (int64_t)k * g.nx;
  return (u[row + ip] - u[cell]) * g.idx + (v[cell + plane] - v[cell]) * g.idy[j] +
         (w[(int64_t)j * plane + (int64_t)kp * g.nx + i] - w[cell]) * g.idz;
}

struct MassPartK {
  GridView g;
  const double* u;
  const double* v;
  const double* w;
  const int64_t* cb;
  const int64_t* count;
  int64_t cap;
  double* partial;
};
template <bool G = false>
__global__ __launch_bounds__(MT) void k_mass_partial(GArg<MassPartK, G> grp_arg_) {
  uint3 bid, gdim;
  const MassPartK& P_ = grp_enter<MassPartK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  GridView g = P_.g;
  const double* __restrict__ u = P_.u;
  const double* __restrict__ v = P_.v;
  const double* __restrict__ w = P_.w;
  const int64_t* __restrict__ cb = P_.cb;
  const int64_t* __restrict__ count = P_.count;
  int64_t cap = P_.cap;
  double* __restrict__ partial = P_.partial;
  __shared__ double sa[MT], sv[MT];
  int64_t n = count[3];
  if (n > cap) n = cap;
  const int64_t chunk = (n + MB - 1) / MB;
  const int64_t lo = bid.x * chunk;
  const int64_t hi = (lo + chunk < n) ? lo + chunk : n;
  double A = 0.0, V = 0.0;
  const double dxdz = g.dx * g.dz;
  for (int64_t f = lo + threadIdx.x; f < hi; f += MT) {
    const int64_t cell = cb[f];
    const int j = (int)(cell / ((int64_t)g.nz * g.nx));
    const double dV = dxdz * g.dy[j];
    A += div_at(g, u, v, w, cell) * dV;
    V += dV;
  }
  sa[threadIdx.x] = A;
  sv[threadIdx.x] = V;
  __syncthreads();
  for (int off = MT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sa[threadIdx.x] += sa[threadIdx.x + off];
      sv[threadIdx.x] += sv[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * bid.x] = sa[0];
    partial[2 * bid.x + 1] = sv[0];
  }
}

struct MassFinK {
  const double* partial;
  const int64_t* count;
  double vtot;
  int use_q;
  double* qf;
  uint32_t* flags;
};
template <bool G = false>
__global__ __launch_bounds__(MB) void k_mass_final(GArg<MassFinK, G> grp_arg_) {
  uint3 bid, gdim;
  const MassFinK& P_ = grp_enter<MassFinK, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  const double* __restrict__ partial = P_.partial;
  const int64_t* __restrict__ count = P_.count;
  double vtot = P_.vtot;
  int use_q = P_.use_q;
  double* __restrict__ qf = P_.qf;
  uint32_t* flags = P_.flags;
  __shared__ double sa[MB], sv[MB];
  sa[threadIdx.x] = partial[2 * threadIdx.x];
  sv[threadIdx.x] = partial[2 * threadIdx.x + 1];
  __syncthreads();
  for (int off = MB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sa[threadIdx.x] += sa[threadIdx.x + off];
      sv[threadIdx.x] += sv[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double q = 0.0;
    if (use_q && count[3] > 0) q = -sa[0] / (vtot - sv[0]);
    if (!isfinite(q)) {
      atomicOr(flags, FLAG_NONFINITE);
      q = 0.0;
    }
    *qf = q;
  }
}

__global__ __launch_bounds__(256) void k_mass_rhs(GridView g, const double* __restrict__ u,
                                                  const double* __restrict__ v,
                                                  const double* __restrict__ w,
                                                  const uint32_t* __restrict__ cb_mask,
                                                  const double* __restrict__ qf, double inv_adt,
                                                  double* __restrict__ rhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const int j = blockIdx.z;
  if (i >= g.nx) return;
  const int64_t cell = ((int64_t)j * g.nz + k) * g.nx + i;
  const double q = *qf;
  rhs[cell] = (cb_mask && test_bit(cb_mask, cell)) ? 0.0
                                                   : (div_at(g, u, v, w, cell) - q) * inv_adt;
}

// Mass- and energy-conserving shape of q_F (paper App. B, Eq. unif_shape):
// q_F = c0 + c1 (p - e) on C_F with r = p - e (e the cell-centred kinetic
// energy of u_hat: each component's square averaged over the two faces),
//   S_i = sum_{C_F} r^i dV, A = sum_{C_B} D u dV, B = sum_{C_B} r D u dV,
//   c0 = (-A S2 + B S1)/C, c1 = (A S1 - B S0)/C, C = S0 S2 - S1^2;
// C vanishes only when r is constant on C_F (the two constraints coincide):
// then the uniform shape c0 = -A/S0, c1 = 0.  The five sums are dense
// (every cell), taken in a fixed two-level order (fixed chunks per block, a
// fixed tree inside each block, then the block partials in order).
constexpr int EB = 512;   // blocks of the first level

__device__ __forceinline__ double kin_at(const GridView& g, const double* u, const double* v,
                                         const double* w, int64_t cell) {
  const int64_t plane = (int64_t)g.nz * g.nx;
  const int i = (int)(cell % g.nx);
  const int k = (int)((cell / g.nx) % g.nz);
  const int j = (int)(cell / plane);
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const int64_t row = (int64_t)j * plane + (int64_t)k * g.nx;
  const double u0 = u[cell], u1 = u[row + ip];
  const double v0 = v[cell], v1 = v[cell + plane];
  const double w0 = w[cell], w1 = w[(int64_t)j * plane + (int64_t)kp * g.nx + i];
  const double eu = 0.5 * (u0 * u0 + u1 * u1);
  const double ev = 0.5 * (v0 * v0 + v1 * v1);
  const double ew = 0.5 * (w0 * w0 + w1 * w1);
  return 0.5 * ((eu + ev) + ew);
}

template <typename T>
__global__ __launch_bounds__(MT) void k_energy_partial(GridView g, const double* __restrict__ u,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ w,
                                                       const T* __restrict__ p,
                                                       const uint32_t* __restrict__ cb_mask,
                                                       double* __restrict__ partial) {
  __shared__ double s[5][MT];
  const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
  const int64_t chunk = (ncell + EB - 1) / EB;
  const int64_t lo = blockIdx.x * chunk;
  const int64_t hi = (lo + chunk < ncell) ? lo + chunk : ncell;
  const int64_t plane = (int64_t)g.nz * g.nx;
  const double dxdz = g.dx * g.dz;
  double S0 = 0.0, S1 = 0.0, S2 = 0.0, A = 0.0, B = 0.0;
  for (int64_t cell = lo + threadIdx.x; cell < hi; cell += MT) {
    const double dV = dxdz * g.dy[(int)(cell / plane)];
    const double r = (double)p[cell] - kin_at(g, u, v, w, cell);
    if (test_bit(cb_mask, cell)) {
      const double D = div_at(g, u, v, w, cell);
      A += D * dV;
      B += (r * D) * dV;
    } else {
      S0 += dV;
      S1 += r * dV;
      S2 += (r * r) * dV;
    }
  }
  s[0][threadIdx.x] = S0;
  s[1][threadIdx.x] = S1;
  s[2][threadIdx.x] = S2;
  s[3][threadIdx.x] = A;
  s[4][threadIdx.x] = B;
  __syncthreads();
  for (int off = MT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int q = 0; q < 5; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 5) partial[5 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(EB) void k_energy_final(const double* __restrict__ partial,
                                                     double* __restrict__ qcoef,
                                                     uint32_t* flags) {
  __shared__ double s[5][EB];
  for (int q = 0; q < 5; ++q) s[q][threadIdx.x] = partial[5 * threadIdx.x + q];
  __syncthreads();
  for (int off = EB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int q = 0; q < 5; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double S0 = s[0][0], S1 = s[1][0], S2 = s[2][0], A = s[3][0], B = s[4][0];
    const double C = S0 * S2 - S1 * S1;
    double c0, c1;
    if (C <= 1e-14 * S0 * S2) {
      c0 = -A / S0;
      c1 = 0.0;
    } else {
      c0 = (-A * S2 + B * S1) / C;
      c1 = (A * S1 - B * S0) / C;
    }
    if (!isfinite(c0) || !isfinite(c1)) {
      atomicOr(flags, FLAG_NONFINITE);
      c0 = 0.0;
      c1 = 0.0;
    }
    qcoef[0] = c0;
    qcoef[1] = c1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_mass_rhs_energy(GridView g, const double* __restrict__ u,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ w,
                                                         const T* __restrict__ p,
                                                         const uint32_t* __restrict__ cb_mask,
                                                         const double* __restrict__ qcoef,
                                                         double inv_adt, double* __restrict__ rhs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const int j = blockIdx.z;
  if (i >= g.nx) return;
  const int64_t cell = ((int64_t)j * g.nz + k) * g.nx + i;
  if (test_bit(cb_mask, cell)) {
    rhs[cell] = 0.0;
    return;
  }
  const double q = qcoef[0] + qcoef[1] * ((double)p[cell] - kin_at(g, u, v, w, cell));
  rhs[cell] = (div_at(g, u, v, w, cell) - q) * inv_adt;
}

void launch_mass_energy(Prof* pf, hipStream_t s, const GridView& g, const double* u,
                        const double* v, const double* w, const void* p, int fp32,
                        const uint32_t* cb_mask, double* partial, double* qcoef,
                        uint32_t* flags) {
  if (fp32)
    IBM_LAUNCH(pf, "mass_energy", s,
               (k_energy_partial<float><<<EB, MT, 0, s>>>(g, u, v, w, (const float*)p, cb_mask,
                                                          partial)));
  else
    IBM_LAUNCH(pf, "mass_energy", s,
               (k_energy_partial<double><<<EB, MT, 0, s>>>(g, u, v, w, (const double*)p,
                                                           cb_mask, partial)));
  IBM_LAUNCH(pf, "mass_final", s, k_energy_final<<<1, EB, 0, s>>>(partial, qcoef, flags));
}

void launch_mass_rhs_energy(Prof* pf, hipStream_t s, const GridView& g, const double* u,
                            const double* v, const double* w, const void* p, int fp32,
                            const uint32_t* cb_mask, const double* qcoef, double inv_adt,
                            double* rhs) {
  dim3 grid((g.nx + 255) / 256, g.nz, g.ny);
  if (fp32)
    IBM_LAUNCH(pf, "mass_rhs", s,
               (k_mass_rhs_energy<float><<<grid, 256, 0, s>>>(g, u, v, w, (const float*)p,
                                                              cb_mask, qcoef, inv_adt, rhs)));
  else
    IBM_LAUNCH(pf, "mass_rhs", s,
               (k_mass_rhs_energy<double><<<grid, 256, 0, s>>>(g, u, v, w, (const double*)p,
                                                               cb_mask, qcoef, inv_adt, rhs)));
}

// Compatibility of the Neumann problem L_c phi = rhs (paper App. A: with
// impermeable walls and periodic x, z the discrete divergence theorem makes
// sum rhs dV vanish for rhs = D u / (alpha dt), the condition for Eq.
// elliptic_mod to have a solution).  Fixed-order sums S = sum rhs dy[j] and
// S_abs = sum |rhs| dy[j] (the factor dx dz cancels): block b takes the rows
// (j, k) of a fixed chunk, its threads stride over x, then fixed trees.
constexpr int CPB = 256;  // blocks of the first level

__global__ __launch_bounds__(MT) void k_compat_partial(GridView g, const double* __restrict__ rhs,
                                                       double* __restrict__ partial) {
  __shared__ double ss[MT], sa[MT];
  const int64_t rows = (int64_t)g.ny * g.nz;
  const int64_t chunk = (rows + CPB - 1) / CPB;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < rows) ? r0 + chunk : rows;
  double S = 0.0, A = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double dyj = g.dy[r / g.nz];
    const double* row = rhs + r * g.nx;
    double s = 0.0, a = 0.0;
    for (int i = threadIdx.x; i < g.nx; i += MT) {
      s += row[i];
      a += fabs(row[i]);
    }
    S += s * dyj;
    A += a * dyj;
  }
  ss[threadIdx.x] = S;
  sa[threadIdx.x] = A;
  __syncthreads();
  for (int off = MT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      ss[threadIdx.x] += ss[threadIdx.x + off];
      sa[threadIdx.x] += sa[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = ss[0];
    partial[2 * blockIdx.x + 1] = sa[0];
  }
}

__global__ __launch_bounds__(CPB) void k_compat_final(const double* __restrict__ partial,
                                                      uint32_t* flags) {
  __shared__ double ss[CPB], sa[CPB];
  ss[threadIdx.x] = partial[2 * threadIdx.x];
  sa[threadIdx.x] = partial[2 * threadIdx.x + 1];
  __syncthreads();
  for (int off = CPB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      ss[threadIdx.x] += ss[threadIdx.x + off];
      sa[threadIdx.x] += sa[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (!(fabs(ss[0]) <= 1e-12 * sa[0])) atomicOr(flags, ss[0] == ss[0] ? FLAG_COMPAT : FLAG_NONFINITE);
  }
}

void launch_compat(Prof* pf, hipStream_t s, const GridView& g, const double* rhs,
                   double* partial, uint32_t* flags) {
  IBM_LAUNCH(pf, "compat", s, k_compat_partial<<<CPB, MT, 0, s>>>(g, rhs, partial));
  IBM_LAUNCH(pf, "compat", s, k_compat_final<<<1, CPB, 0, s>>>(partial, flags));
}

// Post-projection divergence (paper Eq. mod_div: D u = q): max over the
// fluid cells C_F of |D u - q_F| with the uniform q_F of the last mass
// correction; fixed chunks of rows per block, block maxima, then their
// maximum.
__global__ __launch_bounds__(MT) void k_div_partial(GridView g, const double* __restrict__ u,
                                                    const double* __restrict__ v,
                                                    const double* __restrict__ w,
                                                    const uint32_t* __restrict__ cb_mask,
                                                    const double* __restrict__ qf,
                                                    double* __restrict__ partial) {
  __shared__ double sm[MT];
  const int64_t rows = (int64_t)g.ny * g.nz;
  const int64_t chunk = (rows + CPB - 1) / CPB;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < rows) ? r0 + chunk : rows;
  const double q = *qf;
  double m = 0.0;
  for (int64_t r = r0; r < r1; ++r)
    for (int i = threadIdx.x; i < g.nx; i += MT) {
      const int64_t cell = r * g.nx + i;
      if (cb_mask && test_bit(cb_mask, cell)) continue;
      m = fmax(m, fabs(div_at(g, u, v, w, cell) - q));
    }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int off = MT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(CPB) void k_div_final(const double* __restrict__ partial,
                                                   double* __restrict__ out) {
  __shared__ double sm[CPB];
  sm[threadIdx.x] = partial[threadIdx.x];
  __syncthreads();
  for (int off = CPB / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

void launch_divergence(Prof* pf, hipStream_t s, const GridView& g, const double* u,
                       const double* v, const double* w, const uint32_t* cb_mask,
                       const double* qf, double* partial, double* out) {
  IBM_LAUNCH(pf, "divergence", s,
             k_div_partial<<<CPB, MT, 0, s>>>(g, u, v, w, cb_mask, qf, partial));
  IBM_LAUNCH(pf, "divergence", s, k_div_final<<<1, CPB, 0, s>>>(partial, out));
}

void launch_mass(Prof* pf, hipStream_t s, const GridView& g, const double* u, const double* v,
                 const double* w, const int64_t* cb, const int64_t* count, int64_t cap,
                 double vtot, int use_q, double* partial, double* qf, uint32_t* flags) {
  const MassPartK P{g, u, v, w, cb, count, cap, partial};
  IBM_LAUNCH_G(pf, "mass_partial", s, (&k_mass_partial<true>), dim3(MB), dim3(MT), 0, P,
               k_mass_partial<<<MB, MT, 0, s>>>(P));
  const MassFinK F{partial, count, vtot, use_q, qf, flags};
  IBM_LAUNCH_G(pf, "mass_final", s, (&k_mass_final<true>), dim3(1), dim3(MB), 0, F,
               k_mass_final<<<1, MB, 0, s>>>(F));
}

void launch_mass_rhs(Prof* pf, hipStream_t s, const GridView& g, const double* u, const double* v,
                     const double* w, const uint32_t* cb_mask, const double* qf, double inv_adt,
                     double* rhs) {
  dim3 grid((g.nx + 255) / 256, g.nz, g.ny);
  IBM_LAUNCH(pf, "mass_rhs", s,
             k_mass_rhs<<<grid, 256, 0, s>>>(g, u, v, w, cb_mask, qf, inv_adt, rhs));
}

}  // namespace ibm
