// Approximate-factorisation line solves of the predictor (paper Sec. 2:
// "approximate factorization of L, yielding three tridiagonal systems per
// direction"):
//   (I - beta L_x) w1 = R   cyclic in x, constant coefficients
//   (I - beta L_z) w2 = w1  cyclic in z, constant coefficients
//   (I - beta L_y) du = w2  Dirichlet walls, stretched spacing; u <- u + du
// with identity rows on the forcing nodes (the stencil never crosses the
// interface, Sec. 3.1 and Fig. 3).
//
// Partitioned solve (divide and conquer with separators): a line of n rows
// is cut into P balanced segments of at most 16 rows, one per thread, held in
// registers.  Each thread eliminates its interior rows (a forward and a
// backward sweep) so that every interior unknown is an affine function of
// the two separators that bound the segment (its own last row and the
// previous segment's last row).  The separator rows then form a P x P
// tridiagonal system (cyclic for x and z), solved in LDS by one thread per
// line; each thread finally reconstructs its rows.  Every element is read
// once and written once.  Identity rows (a = c = 0, b = 1, d = 0) need no
// special path.
#include "geom.h"

namespace ibm {

constexpr int LMAX = LINE_LMAX;

struct LineK {
  double* d;          // right-hand side in; solution out (x, z)
  double* u;          // y only: u += solution
  const uint32_t* mask;
  double* sa;         // scratch for segments holding identity rows
  double* sc;
  const double* tab;  // mask-free elimination tables [4][P][LMAX]
  int n, P, L, r;     // rows, segments, base length, segments with L+1 rows
  int cyc;
  double a, b, c;     // constant coefficients (x, z)
  const double* A;    // per-row coefficients (y)
  const double* B;
  const double* C;
  int mode;           // 0 x-rows, 1 z-lines, 2 y-lines
  int nx, nz, j0, nj;
  int64_t plane;
  int tl;             // lines per block
};

__device__ __forceinline__ void row_coef(const LineK& K, int i, double& a, double& b, double& c) {
  if (K.A) {
    a = K.A[i];
    b = K.B[i];
    c = K.C[i];
  } else {
    a = K.a;
    b = K.b;
    c = K.c;
  }
}

__device__ __forceinline__ double row_a(const LineK& K, int i) { return K.A ? K.A[i] : K.a; }

// serial solve of one line's P x P cyclic separator system (Sherman-
// Morrison on top of Thomas), for cyclic lines whose segment count is not a
// power of two.  A(f, s) addresses the LDS arrays: f = 3..6 the sub-, main,
// super-diagonal and right-hand side, 7 the solution, 0 and 1 scratch.
template <typename Acc>
__device__ void reduced_solve_cyclic(Acc A, int P) {
  const double g0 = -A(4, 0);
  const double bc = A(3, 0);      // couples z[P-1] in row 0
  const double ac = A(5, P - 1);  // couples z[0] in row P-1
  double cpp = 0.0, yp = 0.0, zp = 0.0;
  for (int s = 0; s < P; ++s) {
    double bs = A(4, s);
    if (s == 0) bs -= g0;
    if (s == P - 1) bs -= ac * bc / g0;
    const double as = s ? A(3, s) : 0.0;
    const double inv = 1.0 / (bs - as * cpp);
    const double us = (s == 0) ? g0 : (s == P - 1 ? ac : 0.0);
    cpp = (s < P - 1) ? A(5, s) * inv : 0.0;
    yp = (A(6, s) - as * yp) * inv;
    zp = (us - as * zp) * inv;
    A(0, s) = cpp;
    A(7, s) = yp;
    A(1, s) = zp;
  }
  for (int s = P - 2; s >= 0; --s) {
    A(7, s) -= A(0, s) * A(7, s + 1);
    A(1, s) -= A(0, s) * A(1, s + 1);
  }
  const double fact = (A(7, 0) + bc * A(7, P - 1) / g0) / (1.0 + A(1, 0) + bc * A(1, P - 1) / g0);
  for (int s = 0; s < P; ++s) A(7, s) -= fact * A(1, s);
}

__global__ __launch_bounds__(256) void k_line(LineK K) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int P = K.P;
  double* tabs = lds;                    // 4 * P * LMAX
  double* sm = lds + 4 * P * LMAX;       // 8 * P * lines per block
  for (int q = tid; q < 4 * P * LMAX; q += blockDim.x) {
    const int qq = q / (P * LMAX), rem = q % (P * LMAX), ss = rem / LMAX, ee = rem % LMAX;
    tabs[(qq * LMAX + ee) * P + ss] = K.tab[q];
  }
  __syncthreads();
  int lb, s;
  if (K.mode == 0) {
    s = tid % P;
    lb = tid / P;
  } else {
    lb = tid % K.tl;
    s = tid / K.tl;
  }
  const bool active = lb < K.tl && s < P;
  // line base offset and element stride
  int64_t base = 0, es = 1;
  bool valid = active;
  if (K.mode == 0) {
    const int64_t line = (int64_t)blockIdx.x * K.tl + lb;
    valid = valid && line < (int64_t)K.nj * K.nz;
    const int j = K.j0 + (int)(line / K.nz), k = (int)(line % K.nz);
    base = ((int64_t)j * K.nz + k) * K.nx;
    es = 1;
  } else {
    const int i = blockIdx.x * K.tl + lb;
    valid = valid && i < K.nx;
    if (K.mode == 1) {
      base = (int64_t)(K.j0 + blockIdx.y) * K.plane + i;
      es = K.nx;
    } else {
      base = (int64_t)K.j0 * K.plane + (int64_t)blockIdx.y * K.nx + i;
      es = K.plane;
    }
  }
  const int lo = s * K.L + (s < K.r ? s : K.r);
  const int len = K.L + (s < K.r ? 1 : 0);
  const int m = len - 1;  // interior rows; row lo+m is the separator
  // table entry (q, e) of this segment; layout [q][e][s] keeps the lanes of
  // consecutive segments on consecutive LDS words
#define TAB(q, e) tabs[((q) * LMAX + (e)) * P + s]
  double dd[LMAX];
  double dz = 0.0, az = 0.0, bz = 1.0, cz = 0.0;
  double a0 = 0.0, c0 = 0.0, ahl = 0.0, chl = 0.0, dhl = 0.0;
  uint32_t mbits = 0;
  if (valid) {
    // issue every load of the segment before using any of them
    double raw[LMAX];
#pragma unroll
    for (int e = 0; e < LMAX; ++e)
      if (e < len) raw[e] = K.d[base + (int64_t)(lo + e) * es];
    if (es == 1) {  // contiguous row: the segment's bits span at most two words
      const int64_t b0 = base + lo;
      const uint32_t w0 = K.mask[b0 >> 5];
      const uint32_t w1 = K.mask[(b0 + len - 1) >> 5];
      const int sh = (int)(b0 & 31);
      const uint64_t both = ((uint64_t)w1 << 32) | w0;
      mbits = (uint32_t)(both >> sh) & ((len >= 32) ? 0xffffffffu : ((1u << len) - 1u));
    } else {
#pragma unroll
      for (int e = 0; e < LMAX; ++e)
        if (e < len) mbits |= (test_bit(K.mask, base + (int64_t)(lo + e) * es) ? 1u : 0u) << e;
    }
#pragma unroll
    for (int e = 0; e < LMAX; ++e)
      if (e < len) {
        const double v = ((mbits >> e) & 1u) ? 0.0 : raw[e];
        if (e < m) dd[e] = v; else dz = v;
      }
    if ((mbits & ((1u << m) - 1u)) == 0u) {
      // mask-free interior: the elimination coefficients come from the tables
      double dt = 0.0;
#pragma unroll
      for (int e = 0; e < LMAX - 1; ++e)
        if (e < m) {
          dt = (dd[e] - row_a(K, lo + e) * dt) * TAB(0, e);
          dd[e] = dt;
        }
      double dh = 0.0;
#pragma unroll
      for (int e = LMAX - 2; e >= 0; --e)
        if (e < m) {
          dh = (e == m - 1) ? dd[e] : dd[e] - TAB(1, e) * dh;
          dd[e] = dh;
          if (e == m - 1) dhl = dh;
        }
      a0 = TAB(2, 0);
      c0 = TAB(3, 0);
      ahl = TAB(2, m - 1);
      chl = TAB(3, m - 1);
    } else {
      // general interior with identity rows: coefficients through the scratch
      double at = 0.0, ct = 0.0, dt = 0.0;
#pragma unroll
      for (int e = 0; e < LMAX - 1; ++e)
        if (e < m) {
          const int i = lo + e;
          const int64_t o = base + (int64_t)i * es;
          double a, b, c;
          row_coef(K, i, a, b, c);
          if ((mbits >> e) & 1u) {
            a = 0.0;
            b = 1.0;
            c = 0.0;
          }
          const double inv = 1.0 / (b - a * ct);
          at = (e == 0) ? a * inv : -a * at * inv;
          ct = c * inv;
          dt = (dd[e] - a * dt) * inv;
          dd[e] = dt;
          K.sa[o] = at;
          K.sc[o] = ct;
        }
      double ah = 0.0, ch = 0.0, dh = 0.0;
#pragma unroll
      for (int e = LMAX - 2; e >= 0; --e)
        if (e < m) {
          const int64_t o = base + (int64_t)(lo + e) * es;
          const double at_e = K.sa[o], ct_e = K.sc[o];
          if (e == m - 1) {
            ah = at_e;
            ch = ct_e;
            dh = dd[e];
            ahl = ah;
            chl = ch;
            dhl = dh;
          } else {
            dh = dd[e] - ct_e * dh;
            ah = at_e - ct_e * ah;
            ch = -ct_e * ch;
          }
          dd[e] = dh;
          K.sa[o] = ah;
          K.sc[o] = ch;
        }
      a0 = ah;
      c0 = ch;
    }
    row_coef(K, lo + m, az, bz, cz);
    if ((mbits >> m) & 1u) {
      az = 0.0;
      bz = 1.0;
      cz = 0.0;
    }
  }
  // LDS: 8 arrays of P doubles per line; neighbouring lanes (consecutive
  // lines in the z/y sweeps, consecutive segments in the x sweep) take
  // consecutive words
  const int TL = K.tl;
  const bool rowmajor = (K.mode == 0);
  auto at = [&](int f, int seg) -> double& {
    return rowmajor ? sm[((size_t)f * TL + lb) * P + seg] : sm[((size_t)f * P + seg) * TL + lb];
  };
  if (active) {
    at(0, s) = a0;
    at(1, s) = c0;
    at(2, s) = valid ? dd[0] : 0.0;
  }
  __syncthreads();
  double ra = 0.0, rb = 1.0, rg = 0.0, rd = 0.0;  // this segment's separator row
  if (active) {
    int sn = s + 1;
    double czz = cz;
    if (sn == P) {
      sn = 0;
      if (!K.cyc) czz = 0.0;
    }
    ra = -az * ahl;
    rb = bz - az * chl - czz * at(0, sn);
    rg = -czz * at(1, sn);
    rd = dz - az * dhl - czz * at(2, sn);
  }
  __syncthreads();
  if (active) {
    at(3, s) = ra;
    at(4, s) = rb;
    at(5, s) = rg;
    at(6, s) = rd;
  }
  __syncthreads();
  if (!K.cyc || (P & (P - 1)) == 0) {
    // parallel cyclic reduction of the separator system, one row per thread;
    // out-of-range rows of a walled line act as identity rows; a cyclic
    // system of 2^k rows closes with couplings onto the row itself
    for (int st = 1; st < P; st <<= 1) {
      double na = 0.0, nb = 1.0, ng = 0.0, nd = 0.0;
      if (active) {
        int im = s - st, ip = s + st;
        double am = 0.0, bm = 1.0, gm = 0.0, dm = 0.0, ap = 0.0, bp = 1.0, gp = 0.0, dp = 0.0;
        if (K.cyc) {
          im &= P - 1;
          ip &= P - 1;
        }
        if (im >= 0) {
          am = at(3, im);
          bm = at(4, im);
          gm = at(5, im);
          dm = at(6, im);
        }
        if (ip < P) {
          ap = at(3, ip);
          bp = at(4, ip);
          gp = at(5, ip);
          dp = at(6, ip);
        }
        const double k1 = ra / bm, k2 = rg / bp;
        na = -am * k1;
        ng = -gp * k2;
        nb = rb - gm * k1 - ap * k2;
        nd = rd - dm * k1 - dp * k2;
      }
      __syncthreads();
      if (active) {
        ra = na;
        rb = nb;
        rg = ng;
        rd = nd;
        at(3, s) = ra;
        at(4, s) = rb;
        at(5, s) = rg;
        at(6, s) = rd;
      }
      __syncthreads();
    }
    if (active) at(7, s) = K.cyc ? rd / (ra + rb + rg) : rd / rb;
  } else {
    if (active && s == 0) reduced_solve_cyclic(at, P);
  }
  __syncthreads();
  if (valid) {
    const double zr = at(7, s);
    const double zl = (s > 0) ? at(7, s - 1) : (K.cyc ? at(7, P - 1) : 0.0);
    const bool fast = (mbits & ((1u << m) - 1u)) == 0u;
#pragma unroll
    for (int e = 0; e < LMAX; ++e)
      if (e < len) {
        const int64_t o = base + (int64_t)(lo + e) * es;
        double x = zr;
        if (e < m) x = fast ? dd[e] - TAB(2, e) * zl - TAB(3, e) * zr
                            : dd[e] - K.sa[o] * zl - K.sc[o] * zr;
        if (K.mode == 2)
          K.u[o] += x;
        else
          K.d[o] = x;
      }
  }
}

static void launch_line(Prof* pf, hipStream_t s, LineK K, const char* name) {
  dim3 grid;
  int threads;
  if (K.mode == 0) {
    K.tl = 256 / K.P;
    threads = K.tl * K.P;
    const int64_t rows = (int64_t)K.nj * K.nz;
    grid = dim3((unsigned)((rows + K.tl - 1) / K.tl));
  } else {
    K.tl = 256 / K.P;
    if (K.tl > 16) K.tl = 16;
    threads = K.tl * K.P;
    grid = dim3((K.nx + K.tl - 1) / K.tl, K.mode == 1 ? K.nj : K.nz);
  }
  const size_t shm = sizeof(double) * (4 * (size_t)K.P * LMAX + 8 * (size_t)K.P * K.tl);
  IBM_LAUNCH(pf, name, s, k_line<<<grid, threads, shm, s>>>(K));
}

static LineK base_k(const GridView& g, double* d, const uint32_t* mask) {
  LineK K{};
  K.d = d;
  K.mask = mask;
  K.nx = g.nx;
  K.nz = g.nz;
  K.plane = (int64_t)g.nz * g.nx;
  return K;
}

void launch_adi_x(Prof* pf, hipStream_t s, const GridView& g, int comp, double* d,
                  const uint32_t* mask, const CyclicTab& t, double* sa, double* sc) {
  LineK K = base_k(g, d, mask);
  K.sa = sa;
  K.sc = sc;
  K.tab = t.seg;
  K.mode = 0;
  K.n = g.nx;
  K.cyc = 1;
  line_plan(K.n, true, &K.P, &K.L, &K.r);
  K.a = t.a;
  K.b = t.b;
  K.c = t.c;
  K.j0 = (comp == 1) ? 1 : 0;
  K.nj = (comp == 1) ? g.ny - 1 : g.ny;
  launch_line(pf, s, K, "adi_x");
}

void launch_adi_z(Prof* pf, hipStream_t s, const GridView& g, int comp, double* d,
                  const uint32_t* mask, const CyclicTab& t, double* sa, double* sc) {
  LineK K = base_k(g, d, mask);
  K.sa = sa;
  K.sc = sc;
  K.tab = t.seg;
  K.mode = 1;
  K.n = g.nz;
  K.cyc = 1;
  line_plan(K.n, true, &K.P, &K.L, &K.r);
  K.a = t.a;
  K.b = t.b;
  K.c = t.c;
  K.j0 = (comp == 1) ? 1 : 0;
  K.nj = (comp == 1) ? g.ny - 1 : g.ny;
  launch_line(pf, s, K, "adi_z");
}

void launch_adi_y(Prof* pf, hipStream_t s, const GridView& g, int comp, double* d, double* u,
                  const uint32_t* mask, const YTab& t, double* sa, double* sc) {
  LineK K = base_k(g, d, mask);
  K.sa = sa;
  K.sc = sc;
  K.tab = t.seg;
  K.mode = 2;
  K.u = u;
  K.n = t.n;
  K.cyc = 0;
  line_plan(K.n, false, &K.P, &K.L, &K.r);
  K.A = t.a;
  K.B = t.b;
  K.C = t.c;
  K.j0 = t.j0;
  K.nj = t.n;
  (void)comp;
  launch_line(pf, s, K, "adi_y");
}

}  // namespace ibm
