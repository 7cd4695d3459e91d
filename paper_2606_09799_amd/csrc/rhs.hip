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
// Every global load of a step is issued one step ahead: the planes of the
// next step, this thread's H_prev values and forcing-mask words.  Vector
// loads complete in issue order, so a load issued late in a step and waited
// for at once would also wait for the whole prefetch; the wall-normal metric
// coefficients of the chunk are therefore staged in LDS at the start.
//
// Storage type T of p, H and R: double, or float in the mixed form.  The
// stencil arithmetic is FP64 in both forms: the velocity is FP64, and
// rounding it to FP32 before differencing would amplify its rounding error by
// 1/spacing; only the results are stored in T.
#include "lanes.h"

namespace ibm {

constexpr int RTX = 64, RTZ = 8;           // tile (threads per block: RTX x RTZ)
constexpr int RHZ = RTZ + 2;                // tile rows with the z halo
constexpr int RJC = 64;  // planes per block at most
// planes per block unless the caller chooses: on 256x192x256 one round of
// blocks on the chip, and 2 halo planes re-read per 48 (measured best of
// 8 .. 48)
constexpr int RJC_DEF = 48;
// ring slots: u 0..2, v 3..5, w 6..8, p 9..10
constexpr int RSLOTS = 11;
// metric coefficients of a chunk after the ring: idy[j0-1 .. j0+JC-1],
// idyc[j0 .. j0+JC], fw0[j0 .. j0+JC], fw1[j0 .. j0+JC]
constexpr int RCN = RJC + 1;
constexpr int RCOEF = 4 * RCN;

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
  int jc;  // planes per block, 1..RJC
};

// Layout of one halo plane in LDS.  Ragged tiles: rows of RTX + 2 values
// (x from i0-1), fetched one value per load.  Whole tiles (nx a multiple of
// RTX): rows of RTX + 4 values (x from i0-2), fetched as aligned pairs, one
// 16-byte load (or 8 for an FP32 pressure) and one 16-byte LDS store per
// pair, which halves the address work of the halo traffic.
template <bool FULL>
struct Halo {
  static constexpr int W = FULL ? 2 : 1;            // values per load
  static constexpr int HX = RTX + (FULL ? 4 : 2);   // values per row
  static constexpr int XO = FULL ? 2 : 1;           // the tile's first column in a row
  static constexpr int PL = HX * RHZ;               // values per plane
  static constexpr int NI = PL / W;                 // loads per plane
  static constexpr int N = (NI + RTX * RTZ - 1) / (RTX * RTZ);  // loads per thread
};
constexpr int RPL_MAX = Halo<true>::PL;  // LDS slot size of either layout

template <typename S, int W> struct PairOf { using type = S; };
template <> struct PairOf<double, 2> { using type = double2; };
template <> struct PairOf<float, 2> { using type = float2; };

// The element at a block-uniform base plus a per-thread 32-bit byte offset,
// the address form that global loads and stores take directly (64-bit base
// in scalar registers, 32-bit vector offset): no 64-bit address per thread
// and field is kept live across the march.  Offsets within one plane stay
// below 2^32 bytes (nx, nz <= 1024).
template <typename X>
__device__ __forceinline__ const X& at_off(const X* base, uint32_t byte_off) {
  return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename X>
__device__ __forceinline__ X& at_off(X* base, uint32_t byte_off) {
  return *reinterpret_cast<X*>(reinterpret_cast<char*>(base) + byte_off);
}

// Offsets within a plane of this thread's loads e = tid + q*threads of the
// tile (i0, k0), with the periodic wrap (grids narrower than a ragged tile
// wrap more than once; a whole tile's pairs start at even x and never
// straddle the wrap); 0 past the tile (read, never stored: the loads stay
// unconditional).  The same for every plane, so computed once per block.
template <bool FULL>
__device__ __forceinline__ void halo_offsets(int (&off)[Halo<FULL>::N], const GridView& g, int i0,
                                             int k0) {
  using H = Halo<FULL>;
#pragma unroll
  for (int q = 0; q < H::N; ++q) {
    const int e = threadIdx.x + q * RTX * RTZ;
    const int lz = e / (H::HX / H::W), lx = (e % (H::HX / H::W)) * H::W;
    int i = i0 - H::XO + lx, k = k0 - 1 + lz;
    i = (i < 0) ? i + g.nx : (i >= g.nx ? (i - g.nx) % g.nx : i);
    k = (k < 0) ? k + g.nz : (k >= g.nz ? (k - g.nz) % g.nz : k);
    off[q] = (e < H::NI) ? k * g.nx + i : 0;
  }
}

// issue the loads of plane j of a field into registers (no wait)
template <bool FULL, typename S>
__device__ __forceinline__ void fetch_plane(double (&r)[Halo<FULL>::N * Halo<FULL>::W],
                                            const S* __restrict__ f, int j, const GridView& g,
                                            const int (&off)[Halo<FULL>::N]) {
  using H = Halo<FULL>;
  const S* fp = f + (int64_t)j * g.nz * g.nx;
#pragma unroll
  for (int q = 0; q < H::N; ++q) {
    const uint32_t ob = (uint32_t)off[q] * (uint32_t)sizeof(S);
    if constexpr (H::W == 2) {
      using P2 = typename PairOf<S, 2>::type;
      const P2 v = at_off(reinterpret_cast<const P2*>(fp), ob);
      r[2 * q] = (double)v.x;
      r[2 * q + 1] = (double)v.y;
    } else {
      r[q] = (double)at_off(fp, ob);
    }
  }
}

// store fetched values into the LDS slot at offset sb
template <bool FULL>
__device__ __forceinline__ void put_plane(double* lds, int sb,
                                          const double (&r)[Halo<FULL>::N * Halo<FULL>::W]) {
  using H = Halo<FULL>;
#pragma unroll
  for (int q = 0; q < H::N; ++q) {
    const int e = threadIdx.x + q * RTX * RTZ;
    if (e < H::NI) {
      if constexpr (H::W == 2)
        *reinterpret_cast<double2*>(lds + sb + 2 * e) = make_double2(r[2 * q], r[2 * q + 1]);
      else
        lds[sb + e] = r[q];
    }
  }
}

// load plane j of a field into the LDS slot at offset sb
template <bool FULL, typename S>
__device__ __forceinline__ void load_plane(double* lds, int sb, const S* __restrict__ f, int j,
                                           const GridView& g, const int (&off)[Halo<FULL>::N]) {
  double r[Halo<FULL>::N * Halo<FULL>::W];
  fetch_plane<FULL>(r, f, j, g, off);
  put_plane<FULL>(lds, sb, r);
}

// Flags of a launch, fixed at compile time so that the march is straight-line
// code: the waits the compiler inserts for the prefetched loads then count
// exactly the loads and stores issued after them.
enum : int {
  RHS_FULL = 1,  // nx and nz are multiples of the tile: every thread owns a cell
  RHS_HPREV = 2, // rho != 0: H_prev is read
  RHS_HOUT = 4,  // H is written (all three components)
};

template <typename T, int F, bool G = false>
__global__ __launch_bounds__(RTX * RTZ) __attribute__((amdgpu_waves_per_eu(4))) void k_rhs(GArg<RhsK<T>, G> grp_arg_) {
  uint3 bid, gdim;
  const RhsK<T>& K = grp_enter<RhsK<T>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  constexpr bool FULL = F & RHS_FULL, HPREV = F & RHS_HPREV, HOUT = F & RHS_HOUT;
  extern __shared__ double lds[];
  const GridView& g = K.g;
  const RhsK<T>& a = K;
  const int nbx = (g.nx + RTX - 1) / RTX, nbz = (g.nz + RTZ - 1) / RTZ;
  const int jc = K.jc;
  const int nchunk = (g.ny + jc - 1) / jc;
  const int64_t t = xcd_tile(bid.x, (int64_t)nbx * nbz * nchunk);
  const int i0 = (int)(t % nbx) * RTX;
  const int k0 = (int)((t / nbx) % nbz) * RTZ;
  const int j0 = (int)(t / ((int64_t)nbx * nbz)) * jc;
  const int j1 = (j0 + jc < g.ny) ? j0 + jc : g.ny;
  const int tx = threadIdx.x % RTX, tz = threadIdx.x / RTX;
  const int i = i0 + tx, k = k0 + tz;
  const bool valid = FULL || (i < g.nx && k < g.nz);
  using H = Halo<FULL>;
  const int lx = tx + H::XO, lz = tz + 1;
  const double idx = g.idx, idz = g.idz;
  const double idx2 = idx * idx, idz2 = idz * idz;
  const double am = a.alpha / a.re;
  const int64_t plane = (int64_t)g.nz * g.nx;
  // value of a ring slot (base offset sb = slot * RPL) at an offset from this
  // thread's cell
  const int me = lz * H::HX + lx;
  auto S = [&](int sb, int dx, int dz) -> double { return lds[sb + me + dz * H::HX + dx]; };
  int off[H::N];
  halo_offsets<FULL>(off, g, i0, k0);
  // the chunk's metric coefficients (only entries the chunk reads)
  double* cf = lds + RSLOTS * H::PL;
  for (int q = threadIdx.x; q < RCOEF; q += RTX * RTZ) {
    const int arr = q / RCN, e = q % RCN;
    double val = 0.0;
    if (arr == 0) {
      const int jj = j0 - 1 + e;
      if (jj >= 0 && jj < j1) val = g.idy[jj];
    } else {
      const int jj = j0 + e;  // <= j1 <= ny
      if (jj <= j1) val = (arr == 1 ? g.idyc : (arr == 2 ? g.fw0 : g.fw1))[jj];
    }
    cf[q] = val;
  }
  // ring slot bases: [0] plane j-1, [1] plane j, [2] plane j+1 (rotated each
  // step); p keeps j-1 and j
  int bu[3], bv[3], bw[3], bp[2];
  for (int q = 0; q < 3; ++q) {
    const int r = (j0 - 1 + q + 3) % 3;
    bu[q] = r * H::PL;
    bv[q] = (3 + r) * H::PL;
    bw[q] = (6 + r) * H::PL;
  }
  for (int q = 0; q < 2; ++q) bp[q] = (9 + (j0 - 1 + q + 2) % 2) * H::PL;
  // ring before the first step: u, v, w at j0-1, j0, j0+1 and p at j0-1, j0
  if (j0 > 0) {
    load_plane<FULL>(lds, bu[0], a.u, j0 - 1, g, off);
    load_plane<FULL>(lds, bv[0], a.v, j0 - 1, g, off);
    load_plane<FULL>(lds, bw[0], a.w, j0 - 1, g, off);
    load_plane<FULL>(lds, bp[0], a.p, j0 - 1, g, off);
  }
  load_plane<FULL>(lds, bu[1], a.u, j0, g, off);
  load_plane<FULL>(lds, bv[1], a.v, j0, g, off);
  load_plane<FULL>(lds, bw[1], a.w, j0, g, off);
  load_plane<FULL>(lds, bp[1], a.p, j0, g, off);
  if (j0 + 1 < g.ny) {
    load_plane<FULL>(lds, bu[2], a.u, j0 + 1, g, off);
    load_plane<FULL>(lds, bw[2], a.w, j0 + 1, g, off);
  }
  load_plane<FULL>(lds, bv[2], a.v, j0 + 1, g, off);  // v has ny+1 planes
  // this thread's column (threads past a ragged edge read the last cell and
  // store nothing)
  const int64_t col = (int64_t)(k < g.nz ? k : g.nz - 1) * g.nx + (i < g.nx ? i : g.nx - 1);
  // the wall planes of v (j = 0 and ny): R = H = 0; plane 0 is also written
  // by the march
  if (j0 == 0 && valid) {
    const int64_t top = (int64_t)g.ny * plane + col;
    a.R[1][top] = (T)0;
    if (HOUT) a.hout[1][top] = (T)0;
  }
  // this thread's H_prev values and mask words of a step, loaded a step ahead
  double hp0 = 0.0, hp1 = 0.0, hp2 = 0.0;
  uint32_t mw0, mw1, mw2;
  // this thread's byte offsets within a plane (cell values and, with whole
  // tiles, whose planes hold a multiple of 32 cells, mask words)
  const uint32_t ocell = (uint32_t)col * (uint32_t)sizeof(T);
  const uint32_t oword = (uint32_t)(col >> 5) * 4u;
  auto fetch_cell = [&](int j) {
    const int64_t pj = (int64_t)j * plane;
    if (FULL) {
      const int64_t wj = pj >> 5;
      mw0 = at_off(a.mask[0] + wj, oword);
      mw1 = at_off(a.mask[1] + wj, oword);
      mw2 = at_off(a.mask[2] + wj, oword);
    } else {
      const int64_t c = pj + col;
      mw0 = a.mask[0][c >> 5];
      mw1 = a.mask[1][c >> 5];
      mw2 = a.mask[2][c >> 5];
    }
    if (HPREV) {
      hp0 = (double)at_off(a.hprev[0] + pj, ocell);
      hp1 = (double)at_off(a.hprev[1] + pj, ocell);
      hp2 = (double)at_off(a.hprev[2] + pj, ocell);
    }
  };
  // software pipeline: the planes of the next step (u, v, w at j+2 and p at
  // j+1) are in flight in registers while plane j is computed.  The loads are
  // unconditional (plane indices clamped; a clamped plane is never stored),
  // so every step issues the same loads in the same order.
  double nu[H::N * H::W], nv[H::N * H::W], nw[H::N * H::W], np[H::N * H::W];
  auto fetch_next = [&](int j) {
    const int ju = (j + 2 < g.ny) ? j + 2 : g.ny - 1;
    const int jv = (j + 2 <= g.ny) ? j + 2 : g.ny;
    const int jp = (j + 1 < g.ny) ? j + 1 : g.ny - 1;
    fetch_plane<FULL>(nu, a.u, ju, g, off);
    fetch_plane<FULL>(nw, a.w, ju, g, off);
    fetch_plane<FULL>(nv, a.v, jv, g, off);
    fetch_plane<FULL>(np, a.p, jp, g, off);
  };
  fetch_cell(j0);
  fetch_next(j0);
  __syncthreads();
  for (int j = j0; j < j1; ++j) {
    const int64_t pj = (int64_t)j * plane;
    const int cj = j - j0;
    const double idyj = cf[cj + 1];
    const bool has_s = j > 0, has_n = j + 1 < g.ny;
    const double ic_n = cf[RCN + cj + 1], ic_s = cf[RCN + cj];
    // weights of the face interpolations at faces j+1 (north) and j (south)
    const double n0 = cf[2 * RCN + cj + 1], n1 = cf[3 * RCN + cj + 1];
    const double s0 = cf[2 * RCN + cj], s1 = cf[3 * RCN + cj];
    const int U0 = bu[1], Um = bu[0], Up = bu[2];
    const int V0 = bv[1], Vm = bv[0], Vp = bv[2];
    const int W0 = bw[1], Wm = bw[0], Wp = bw[2];
    const int P0 = bp[1], Pm = bp[0];
    const uint32_t bit = FULL ? (uint32_t)(col & 31) : (uint32_t)((pj + col) & 31);
    double r_u, r_v = 0.0, r_w, h_u, h_v = 0.0, h_w;
    // ---------------------------------------------------------- u node
    {
      const double uc = S(U0, 0, 0), ue = S(U0, 1, 0), uw = S(U0, -1, 0);
      const double ut = S(U0, 0, 1), ub = S(U0, 0, -1);
      const double un = has_n ? S(Up, 0, 0) : 0.0;
      const double us = has_s ? S(Um, 0, 0) : 0.0;
      const double bp_ = 0.5 * (uc + ue), bm = 0.5 * (uw + uc);
      const double tx_ = (bp_ * bp_ - bm * bm) * idx;
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
      if (HPREV) r += a.rho * hp0;
      h_u = H;
      r_u = ((mw0 >> bit) & 1u) ? 0.0 : a.dt * r;
    }
    // ---------------------------------------------------------- w node
    {
      const double wc = S(W0, 0, 0), we = S(W0, 1, 0), ww = S(W0, -1, 0);
      const double wt = S(W0, 0, 1), wb = S(W0, 0, -1);
      const double wn = has_n ? S(Wp, 0, 0) : 0.0;
      const double ws = has_s ? S(Wm, 0, 0) : 0.0;
      const double bp_ = 0.5 * (wc + wt), bm = 0.5 * (wb + wc);
      const double tz = (bp_ * bp_ - bm * bm) * idz;
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
      if (HPREV) r += a.rho * hp2;
      h_w = H;
      r_w = ((mw2 >> bit) & 1u) ? 0.0 : a.dt * r;
    }
    // ---------------------------------------------------- v node (face j)
    if (j > 0) {  // face 0 is the wall: R = H = 0
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
                       ((vn - vc) * idyj - (vc - vs) * cf[cj]) * ic_s;
      const double gp = (S(P0, 0, 0) - S(Pm, 0, 0)) * ic_s;
      double r = a.gamma * H - a.alpha * gp + am * L;
      if (HPREV) r += a.rho * hp1;
      h_v = H;
      r_v = ((mw1 >> bit) & 1u) ? 0.0 : a.dt * r;
    }
    if (valid) {
      at_off(a.R[0] + pj, ocell) = (T)r_u;
      at_off(a.R[2] + pj, ocell) = (T)r_w;
      at_off(a.R[1] + pj, ocell) = (T)r_v;
      if (HOUT) {
        at_off(a.hout[0] + pj, ocell) = (T)h_u;
        at_off(a.hout[2] + pj, ocell) = (T)h_w;
        at_off(a.hout[1] + pj, ocell) = (T)h_v;
      }
    }
    if (j + 1 < j1) {
      __syncthreads();  // every read of the slots of j-1 is done
      // rotate: the slots of j-1 take the planes of j+2 (p: j-1 takes j+1)
      int t_ = bu[0]; bu[0] = bu[1]; bu[1] = bu[2]; bu[2] = t_;
      t_ = bv[0]; bv[0] = bv[1]; bv[1] = bv[2]; bv[2] = t_;
      t_ = bw[0]; bw[0] = bw[1]; bw[1] = bw[2]; bw[2] = t_;
      t_ = bp[0]; bp[0] = bp[1]; bp[1] = t_;
      if (j + 2 < g.ny) {
        put_plane<FULL>(lds, bu[2], nu);
        put_plane<FULL>(lds, bw[2], nw);
      }
      if (j + 2 <= g.ny) put_plane<FULL>(lds, bv[2], nv);
      put_plane<FULL>(lds, bp[1], np);
      fetch_cell(j + 1);
      fetch_next(j + 1);
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
  K.jc = (a.planes >= 1 && a.planes <= RJC) ? a.planes : RJC_DEF;
  const int64_t blocks = (int64_t)((g.nx + RTX - 1) / RTX) * ((g.nz + RTZ - 1) / RTZ) *
                         ((g.ny + K.jc - 1) / K.jc);
  const size_t shm = sizeof(double) * (RSLOTS * RPL_MAX + RCOEF);
  const int f = ((g.nx % RTX == 0 && g.nz % RTZ == 0) ? RHS_FULL : 0) |
                (a.rho != 0.0 ? RHS_HPREV : 0) |
                ((a.hout[0] && a.hout[1] && a.hout[2]) ? RHS_HOUT : 0);
  // H written per component when only some are requested: none here (the
  // host passes all three or none), checked by the caller
  switch (f) {
#define RHS_CASE(F_)                                                              \
  case F_:                                                                        \
    IBM_LAUNCH_G(pf, "rhs", s, (&k_rhs<T, F_, true>), dim3((unsigned)blocks), dim3(RTX * RTZ), shm, \
                 K, k_rhs<T, F_><<<(unsigned)blocks, RTX * RTZ, shm, s>>>(K));           \
    break;
    RHS_CASE(0) RHS_CASE(1) RHS_CASE(2) RHS_CASE(3)
    RHS_CASE(4) RHS_CASE(5) RHS_CASE(6) RHS_CASE(7)
#undef RHS_CASE
  }
}

void launch_rhs(Prof* pf, hipStream_t s, const GridView& g, const RhsArgs& a) {
  if (a.fp32)
    run_rhs<float>(pf, s, g, a);
  else
    run_rhs<double>(pf, s, g, a);
}

// Volume force of one component (the forces that Sec. 4.2 and 4.3 add to
// Eq. NS_prov), added to the right-hand side the RHS pass wrote:
// R += alpha dt (f0 + kappa u) on the component's unknown nodes [lo, hi)
// that are not forcing nodes, in FP64 arithmetic.
template <typename T>
__global__ __launch_bounds__(256) void k_vforce(int64_t lo, int64_t hi, T* __restrict__ R,
                                                const uint32_t* __restrict__ mask,
                                                const double* __restrict__ u,
                                                const double* __restrict__ f0,
                                                const double* __restrict__ kap, double adt) {
  const int64_t i = lo + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= hi || test_bit(mask, i)) return;
  double f = f0 ? f0[i] : 0.0;
  if (kap) f += kap[i] * u[i];
  R[i] = (T)((double)R[i] + adt * f);
}

void launch_vforce(Prof* pf, hipStream_t s, const GridView& g, int comp, void* R, int fp32,
                   const uint32_t* mask, const double* u, const double* f0, const double* kappa,
                   double adt) {
  const int64_t plane = (int64_t)g.nz * g.nx;
  const int64_t lo = (comp == 1) ? plane : 0, hi = (int64_t)g.ny * plane;  // v: interior faces
  const unsigned blocks = (unsigned)((hi - lo + 255) / 256);
  if (fp32)
    IBM_LAUNCH(pf, "vforce", s,
               (k_vforce<float><<<blocks, 256, 0, s>>>(lo, hi, (float*)R, mask, u, f0, kappa, adt)));
  else
    IBM_LAUNCH(pf, "vforce", s,
               (k_vforce<double><<<blocks, 256, 0, s>>>(lo, hi, (double*)R, mask, u, f0, kappa,
                                                        adt)));
}

}  // namespace ibm
