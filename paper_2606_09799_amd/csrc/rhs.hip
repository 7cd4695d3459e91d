// Explicit right-hand side of the predictor (paper Eq. NS_prov in delta form):
//   R = dt [gamma H(u) + rho H_prev - alpha (G p - f) + (alpha/Re) L u]
// on the fluid nodes, R = 0 on the forcing nodes (Eq. IB_step: those nodes
// are not predicted) and on the v wall planes.  H = -div(u u) in flux
// (conservative) form; L the viscous Laplacian with the wall value 0 at half
// a cell from the first centre; G p the staggered pressure gradient; f the
// constant driving force along x.
//
// LDS-tiled wall-normal march.  A block owns a tile of TX x TZ (x, z) columns
// and a chunk of JC planes.  It keeps a ring of planes in LDS, each with a
// one-cell halo in x and z (periodic wrap): u, v and w at j-1, j, j+1 and p
// at j-1, j.  Each step loads the next plane of u, v, w and the current
// plane of p (coalesced, every value once per block), then every thread
// computes the three components of its (i, j, k) from LDS.  The stencil's
// ~50 neighbour reads thus cost LDS reads instead of vector-memory
// instructions, which otherwise saturate the address units.
//
// Storage type T of p, H and R: double, or float in the mixed form.  The
// stencil arithmetic is FP64 in both forms: the velocity is FP64, and
// rounding it to FP32 before differencing would amplify its rounding error by
// 1/spacing; only the results are stored in T.
#include "geom.h"

namespace ibm {

constexpr int RTX = 64, RTZ = 8;           // tile (threads per block: RTX x RTZ)
constexpr int RHX = RTX + 2, RHZ = RTZ + 2; // tile with halo
constexpr int RPL = RHX * RHZ;              // values per plane in LDS
constexpr int RJC = 16;                     // planes per block
// ring slots: u 0..2, v 3..5, w 6..8, p 9..10
constexpr int RSLOTS = 11;

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

// elements of one halo plane per thread (RPL values over RTX*RTZ threads)
constexpr int RPT = (RPL + RTX * RTZ - 1) / (RTX * RTZ);

// Offsets within a plane of this thread's halo elements e = tid + q*threads
// of the tile (i0, k0), with the periodic wrap (i >= -1 and k >= -1; grids
// narrower than the tile wrap more than once); -1 past the tile.  The same
// for every plane, so computed once per block.
__device__ __forceinline__ void halo_offsets(int (&off)[RPT], const GridView& g, int i0, int k0) {
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int e = threadIdx.x + q * RTX * RTZ;
    const int lz = e / RHX, lx = e % RHX;
    int i = i0 - 1 + lx, k = k0 - 1 + lz;
    i = (i < 0) ? i + g.nx : (i >= g.nx ? (i - g.nx) % g.nx : i);
    k = (k < 0) ? k + g.nz : (k >= g.nz ? (k - g.nz) % g.nz : k);
    off[q] = (e < RPL) ? k * g.nx + i : -1;
  }
}

// issue the loads of plane j of a field into registers (no wait)
template <typename S>
__device__ __forceinline__ void fetch_plane(double (&r)[RPT], const S* __restrict__ f, int j,
                                            const GridView& g, const int (&off)[RPT]) {
  const S* fp = f + (int64_t)j * g.nz * g.nx;
#pragma unroll
  for (int q = 0; q < RPT; ++q) r[q] = (off[q] >= 0) ? (double)fp[off[q]] : 0.0;
}

// load plane j of a field into LDS slot `slot`
template <typename S>
__device__ __forceinline__ void load_plane(double* lds, int slot, const S* __restrict__ f, int j,
                                           const GridView& g, const int (&off)[RPT]) {
  const S* fp = f + (int64_t)j * g.nz * g.nx;
#pragma unroll
  for (int q = 0; q < RPT; ++q)
    if (off[q] >= 0) lds[slot * RPL + threadIdx.x + q * RTX * RTZ] = (double)fp[off[q]];
}

__device__ __forceinline__ void put_plane(double* lds, int slot, const double (&r)[RPT]) {
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int e = threadIdx.x + q * RTX * RTZ;
    if (e < RPL) lds[slot * RPL + e] = r[q];
  }
}

template <typename T>
__global__ __launch_bounds__(RTX * RTZ) void k_rhs(RhsK<T> K) {
  extern __shared__ double lds[];
  const GridView& g = K.g;
  const RhsK<T>& a = K;
  const int nbx = (g.nx + RTX - 1) / RTX, nbz = (g.nz + RTZ - 1) / RTZ;
  const int nchunk = (g.ny + RJC - 1) / RJC;
  const int64_t t = xcd_tile(blockIdx.x, (int64_t)nbx * nbz * nchunk);
  const int i0 = (int)(t % nbx) * RTX;
  const int k0 = (int)((t / nbx) % nbz) * RTZ;
  const int j0 = (int)(t / ((int64_t)nbx * nbz)) * RJC;
  const int j1 = (j0 + RJC < g.ny) ? j0 + RJC : g.ny;
  const int tx = threadIdx.x % RTX, tz = threadIdx.x / RTX;
  const int i = i0 + tx, k = k0 + tz;
  const bool valid = i < g.nx && k < g.nz;
  const int lx = tx + 1, lz = tz + 1;
  const double idx = g.idx, idz = g.idz;
  const double idx2 = idx * idx, idz2 = idz * idz;
  const double am = a.alpha / a.re;
  const int64_t plane = (int64_t)g.nz * g.nx;
  // value of a ring slot at an offset from this thread's cell
  auto S = [&](int slot, int dx, int dz) -> double {
    return lds[slot * RPL + (lz + dz) * RHX + (lx + dx)];
  };
  auto su = [](int jj) { return (jj + 3) % 3; };
  auto sv = [](int jj) { return 3 + (jj + 3) % 3; };
  auto sw = [](int jj) { return 6 + (jj + 3) % 3; };
  auto sp = [](int jj) { return 9 + (jj + 2) % 2; };
  int off[RPT];
  halo_offsets(off, g, i0, k0);
  // ring before the first step: u, v, w at j0-1, j0, j0+1 and p at j0-1, j0
  if (j0 > 0) {
    load_plane(lds, su(j0 - 1), a.u, j0 - 1, g, off);
    load_plane(lds, sv(j0 - 1), a.v, j0 - 1, g, off);
    load_plane(lds, sw(j0 - 1), a.w, j0 - 1, g, off);
    load_plane(lds, sp(j0 - 1), a.p, j0 - 1, g, off);
  }
  load_plane(lds, su(j0), a.u, j0, g, off);
  load_plane(lds, sv(j0), a.v, j0, g, off);
  load_plane(lds, sw(j0), a.w, j0, g, off);
  load_plane(lds, sp(j0), a.p, j0, g, off);
  if (j0 + 1 < g.ny) {
    load_plane(lds, su(j0 + 1), a.u, j0 + 1, g, off);
    load_plane(lds, sw(j0 + 1), a.w, j0 + 1, g, off);
  }
  load_plane(lds, sv(j0 + 1), a.v, j0 + 1, g, off);  // v has ny+1 planes
  // software pipeline: the planes of the next step (u, v, w at j+2 and p at
  // j+1) are in flight in registers while plane j is computed
  double nu[RPT], nv[RPT], nw[RPT], np[RPT];
  auto fetch_next = [&](int j) {
    if (j + 2 < g.ny) {
      fetch_plane(nu, a.u, j + 2, g, off);
      fetch_plane(nw, a.w, j + 2, g, off);
    }
    if (j + 2 <= g.ny) fetch_plane(nv, a.v, j + 2, g, off);
    if (j + 1 < g.ny) fetch_plane(np, a.p, j + 1, g, off);
  };
  if (j0 + 1 < j1) fetch_next(j0);
  __syncthreads();
  for (int j = j0; j < j1; ++j) {
    if (valid) {
      const int64_t c = (int64_t)j * plane + (int64_t)k * g.nx + i;
      const double idyj = g.idy[j];
      const bool has_s = j > 0, has_n = j + 1 < g.ny;
      const double ic_n = g.idyc[j + 1], ic_s = g.idyc[j];
      // weights of the face interpolations at faces j+1 (north) and j (south)
      const double n0 = g.fw0[j + 1], n1 = g.fw1[j + 1], s0 = g.fw0[j], s1 = g.fw1[j];
      const int U0 = su(j), Um = su(j - 1), Up = su(j + 1);
      const int V0 = sv(j), Vm = sv(j - 1), Vp = sv(j + 1);
      const int W0 = sw(j), Wm = sw(j - 1), Wp = sw(j + 1);
      const int P0 = sp(j), Pm = sp(j - 1);
      // ---------------------------------------------------------- u node
      {
        const double uc = S(U0, 0, 0), ue = S(U0, 1, 0), uw = S(U0, -1, 0);
        const double ut = S(U0, 0, 1), ub = S(U0, 0, -1);
        const double un = has_n ? S(Up, 0, 0) : 0.0;
        const double us = has_s ? S(Um, 0, 0) : 0.0;
        const double bp = 0.5 * (uc + ue), bm = 0.5 * (uw + uc);
        const double tx_ = (bp * bp - bm * bm) * idx;
        const double iyn = has_n ? uc * n0 + un * n1 : 0.0;
        const double iys = has_s ? us * s0 + uc * s1 : 0.0;
        const double vn = 0.5 * (S(Vp, -1, 0) + S(Vp, 0, 0));
        const double vs = 0.5 * (S(V0, -1, 0) + S(V0, 0, 0));
        const double ty = (iyn * vn - iys * vs) * idyj;
        const double fzp = (0.5 * (uc + ut)) * (0.5 * (S(W0, -1, 1) + S(W0, 0, 1)));
        const double fzm = (0.5 * (ub + uc)) * (0.5 * (S(W0, -1, 0) + S(W0, 0, 0)));
        const double tz = (fzp - fzm) * idz;
        const double H = -(tx_ + ty + tz);
        const double L = ((ue - uc) - (uc - uw)) * idx2 + ((ut - uc) - (uc - ub)) * idz2 +
                         ((un - uc) * ic_n - (uc - us) * ic_s) * idyj;
        const double gp = (S(P0, 0, 0) - S(P0, -1, 0)) * idx;
        double r = a.gamma * H - a.alpha * (gp - a.fx) + am * L;
        if (a.rho != 0.0) r += a.rho * (double)a.hprev[0][c];
        if (a.hout[0]) a.hout[0][c] = (T)H;
        a.R[0][c] = (T)(test_bit(a.mask[0], c) ? 0.0 : a.dt * r);
      }
      // ---------------------------------------------------------- w node
      {
        const double wc = S(W0, 0, 0), we = S(W0, 1, 0), ww = S(W0, -1, 0);
        const double wt = S(W0, 0, 1), wb = S(W0, 0, -1);
        const double wn = has_n ? S(Wp, 0, 0) : 0.0;
        const double ws = has_s ? S(Wm, 0, 0) : 0.0;
        const double bp = 0.5 * (wc + wt), bm = 0.5 * (wb + wc);
        const double tz = (bp * bp - bm * bm) * idz;
        const double iyn = has_n ? wc * n0 + wn * n1 : 0.0;
        const double iys = has_s ? ws * s0 + wc * s1 : 0.0;
        const double vn = 0.5 * (S(Vp, 0, -1) + S(Vp, 0, 0));
        const double vs = 0.5 * (S(V0, 0, -1) + S(V0, 0, 0));
        const double ty = (iyn * vn - iys * vs) * idyj;
        const double fxp = (0.5 * (wc + we)) * (0.5 * (S(U0, 1, -1) + S(U0, 1, 0)));
        const double fxm = (0.5 * (ww + wc)) * (0.5 * (S(U0, 0, -1) + S(U0, 0, 0)));
        const double tx_ = (fxp - fxm) * idx;
        const double H = -(tx_ + ty + tz);
        const double L = ((we - wc) - (wc - ww)) * idx2 + ((wt - wc) - (wc - wb)) * idz2 +
                         ((wn - wc) * ic_n - (wc - ws) * ic_s) * idyj;
        const double gp = (S(P0, 0, 0) - S(P0, 0, -1)) * idz;
        double r = a.gamma * H - a.alpha * gp + am * L;
        if (a.rho != 0.0) r += a.rho * (double)a.hprev[2][c];
        if (a.hout[2]) a.hout[2][c] = (T)H;
        a.R[2][c] = (T)(test_bit(a.mask[2], c) ? 0.0 : a.dt * r);
      }
      // ---------------------------------------------------- v node (face j)
      if (j == 0) {
        const int64_t top = (int64_t)g.ny * plane + (int64_t)k * g.nx + i;
        a.R[1][c] = (T)0;  // wall planes
        a.R[1][top] = (T)0;
        if (a.hout[1]) {
          a.hout[1][c] = (T)0;
          a.hout[1][top] = (T)0;
        }
      } else {
        const double vc = S(V0, 0, 0), ve = S(V0, 1, 0), vw = S(V0, -1, 0);
        const double vt = S(V0, 0, 1), vb = S(V0, 0, -1);
        const double vn = S(Vp, 0, 0), vs = S(Vm, 0, 0);
        const double uy_i = S(Um, 0, 0) * s0 + S(U0, 0, 0) * s1;
        const double uy_ip = S(Um, 1, 0) * s0 + S(U0, 1, 0) * s1;
        const double tx_ = (uy_ip * (0.5 * (vc + ve)) - uy_i * (0.5 * (vw + vc))) * idx;
        const double ct = 0.5 * (vc + vn), cs = 0.5 * (vs + vc);
        const double ty = (ct * ct - cs * cs) * ic_s;
        const double wy_k = S(Wm, 0, 0) * s0 + S(W0, 0, 0) * s1;
        const double wy_kp = S(Wm, 0, 1) * s0 + S(W0, 0, 1) * s1;
        const double tz = (wy_kp * (0.5 * (vc + vt)) - wy_k * (0.5 * (vb + vc))) * idz;
        const double H = -(tx_ + ty + tz);
        const double L = ((ve - vc) - (vc - vw)) * idx2 + ((vt - vc) - (vc - vb)) * idz2 +
                         ((vn - vc) * idyj - (vc - vs) * g.idy[j - 1]) * ic_s;
        const double gp = (S(P0, 0, 0) - S(Pm, 0, 0)) * ic_s;
        double r = a.gamma * H - a.alpha * gp + am * L;
        if (a.rho != 0.0) r += a.rho * (double)a.hprev[1][c];
        if (a.hout[1]) a.hout[1][c] = (T)H;
        a.R[1][c] = (T)(test_bit(a.mask[1], c) ? 0.0 : a.dt * r);
      }
    }
    if (j + 1 < j1) {
      __syncthreads();  // every read of the slots of j-1 is done
      if (j + 2 < g.ny) {
        put_plane(lds, su(j + 2), nu);
        put_plane(lds, sw(j + 2), nw);
      }
      if (j + 2 <= g.ny) put_plane(lds, sv(j + 2), nv);
      put_plane(lds, sp(j + 1), np);
      if (j + 2 < j1) fetch_next(j + 1);
      __syncthreads();
    }
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
  const int64_t blocks = (int64_t)((g.nx + RTX - 1) / RTX) * ((g.nz + RTZ - 1) / RTZ) *
                         ((g.ny + RJC - 1) / RJC);
  const size_t shm = sizeof(double) * RSLOTS * RPL;
  IBM_LAUNCH(pf, "rhs", s, k_rhs<T><<<(unsigned)blocks, RTX * RTZ, shm, s>>>(K));
}

void launch_rhs(Prof* pf, hipStream_t s, const GridView& g, const RhsArgs& a) {
  if (a.fp32)
    run_rhs<float>(pf, s, g, a);
  else
    run_rhs<double>(pf, s, g, a);
}

}  // namespace ibm
