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
//
// Precision T: double, or float in the mixed form (right-hand sides,
// tables, scratch and arithmetic in FP32; the y sweep adds its FP32 solution
// to the FP64 velocity).
#include "lanes.h"

namespace ibm {

constexpr int LMAX = LINE_LMAX;

template <typename T>
struct LineK {
  T* d;               // right-hand side in; solution out (x, z)
  double* u;          // y only: u += solution
  const uint32_t* mask;
  T* sa;              // scratch for segments holding identity rows
  T* sc;
  const T* tab;       // mask-free elimination tables [LINE_NTAB][P][LINE_TLD]
  int n, P, L, r;     // rows, segments, base length, segments with L+1 rows
  int cyc;
  T a, b, c;          // constant coefficients (x, z)
  const T* A;         // per-row coefficients (y)
  const T* B;
  const T* C;
  int mode;           // 0 x-rows, 1 z-lines, 2 y-lines
  int tab1;           // every segment has the same table (constant
                      // coefficients, equal segments): only segment 0's is staged
  int nx, nz, j0, nj;
  int64_t plane;
  int tl;             // lines per block
  int PP;             // column sweeps: P rounded up to a power of two
  int xrow;           // y sweep, register kernel: whole z rows per XCD (1-D
                      // grid) rather than z-major blocks (2-D grid)
};

template <typename T>
__device__ __forceinline__ void row_coef(const LineK<T>& K, int i, T& a, T& b, T& c) {
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


// serial solve of one line's P x P cyclic separator system (Sherman-
// Morrison on top of Thomas), for cyclic lines whose segment count is not a
// power of two.  A(f, s) addresses the LDS arrays: f = 3..6 the sub-, main,
// super-diagonal and right-hand side, 7 the solution, 0 and 1 scratch.
template <typename T, typename Acc>
__device__ void reduced_solve_cyclic(Acc A, int P) {
  const T g0 = -A(4, 0);
  const T bc = A(3, 0);      // couples z[P-1] in row 0
  const T ac = A(5, P - 1);  // couples z[0] in row P-1
  T cpp = 0, yp = 0, zp = 0;
  for (int s = 0; s < P; ++s) {
    T bs = A(4, s);
    if (s == 0) bs -= g0;
    if (s == P - 1) bs -= ac * bc / g0;
    const T as = s ? A(3, s) : T(0);
    const T inv = T(1) / (bs - as * cpp);
    const T us = (s == 0) ? g0 : (s == P - 1 ? ac : T(0));
    cpp = (s < P - 1) ? A(5, s) * inv : T(0);
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
  const T fact = (A(7, 0) + bc * A(7, P - 1) / g0) / (T(1) + A(1, 0) + bc * A(1, P - 1) / g0);
  for (int s = 0; s < P; ++s) A(7, s) -= fact * A(1, s);
}

// MODE: 0 x rows, 1 z lines, 2 y lines (compile time, so each instance
// carries only its own addressing).  FIXED: every segment holds exactly LMAX
// rows (n = P * LMAX), so the segment loops have no runtime bounds.
template <typename T, int MODE, bool FIXED, bool G = false>
__global__ __launch_bounds__(MODE == 0 ? 256 : 1024) void k_line(GArg<LineK<T>, G> grp_arg_) {
  uint3 bid, gdim;
  const LineK<T>& K = grp_enter<LineK<T>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  extern __shared__ __align__(16) unsigned char ldsraw[];
  T* lds = reinterpret_cast<T*>(ldsraw);
  const int tid = threadIdx.x;
  const int P = K.P;
  const int tP = K.tab1 ? 1 : P;         // segments in the staged tables
  T* tabs = lds;                         // LINE_NTAB * tP * LMAX
  T* sm = lds + LINE_NTAB * tP * LMAX;   // 8 * P * lines per block
  // x sweep: the block's rows are staged through LDS (coalesced loads and
  // stores; each thread then reads its segment from LDS), one pad slot every
  // 16 values so that consecutive segments fall on different banks; the row
  // buffer is reused for the separator arrays once the rows are in registers
  T* rowbuf = sm;
  const int RS = K.n + (K.n >> 4) + 1;
  // tables [q][e][s] from the host layout [q][s][e], written in LDS order
  // (consecutive lanes on consecutive words)
  for (int q = tid; q < LINE_NTAB * tP * LMAX; q += blockDim.x) {
    const int qe = q / tP, ss = q % tP, qq = qe / LMAX, ee = qe % LMAX;
    tabs[q] = K.tab[((size_t)qq * P + ss) * LINE_TLD + ee];
  }
  __syncthreads();
  int lb, s;
  if (MODE == 0) {
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
  if (MODE == 0) {
    const int64_t line = (int64_t)bid.x * K.tl + lb;
    valid = valid && line < (int64_t)K.nj * K.nz;
    const int j = K.j0 + (int)(line / K.nz), k = (int)(line % K.nz);
    base = ((int64_t)j * K.nz + k) * K.nx;
    es = 1;
  } else {
    const int i = bid.x * K.tl + lb;
    valid = valid && i < K.nx;
    if (MODE == 1) {
      base = (int64_t)(K.j0 + bid.y) * K.plane + i;
      es = K.nx;
    } else {
      base = (int64_t)K.j0 * K.plane + (int64_t)bid.y * K.nx + i;
      es = K.plane;
    }
  }
  const int lo = FIXED ? s * LMAX : s * K.L + (s < K.r ? s : K.r);
  const int len = FIXED ? LMAX : K.L + (s < K.r ? 1 : 0);
  const int m = len - 1;  // interior rows; row lo+m is the separator
  // x sweep: rows of this block and their staging
  int xrows = 0;
  const T* xsrc = nullptr;
  if (MODE == 0) {
    const int64_t l0 = (int64_t)bid.x * K.tl;
    const int64_t nl = (int64_t)K.nj * K.nz;
    xrows = (int)((l0 + K.tl <= nl) ? K.tl : nl - l0);
    xsrc = K.d + ((int64_t)K.j0 * K.nz + l0) * K.n;
    // the block's rows are consecutive in memory: one flat, coalesced pass
    // over all of them (short rows would leave most threads idle row by row)
    for (int e = tid; e < xrows * K.n; e += blockDim.x) {
      const int r = e / K.n, c = e - r * K.n;
      rowbuf[r * RS + c + (c >> 4)] = xsrc[e];
    }
    __syncthreads();
  }
  auto xpos = [&](int e) { return lb * RS + (lo + e) + ((lo + e) >> 4); };
  // table entry (q, e) of this segment; layout [q][e][s] keeps the lanes of
  // consecutive segments on consecutive LDS words
  const int ts = K.tab1 ? 0 : s;
#define TAB(q, e) tabs[((q) * LMAX + (e)) * tP + ts]
  T dd[LMAX];
  double uu[MODE == 2 ? LMAX : 1];
  T dz = 0, az = 0, bz = 1, cz = 0;
  T a0 = 0, c0 = 0, ahl = 0, chl = 0, dhl = 0;
  uint32_t mbits = 0;
  if (valid) {
    // issue every load of the segment before using any of them
    T raw[LMAX];
#pragma unroll
    for (int e = 0; e < LMAX; ++e)
      if (e < len) raw[e] = (MODE == 0) ? rowbuf[xpos(e)] : K.d[base + (int64_t)(lo + e) * es];
    if (MODE == 2) {
      // the velocity the solution is added to, loaded now so that its
      // latency overlaps the solve
#pragma unroll
      for (int e = 0; e < LMAX; ++e)
        if (e < len) uu[e] = K.u[base + (int64_t)(lo + e) * es];
    }
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
        const T v = ((mbits >> e) & 1u) ? T(0) : raw[e];
        if (e < m) dd[e] = v; else dz = v;
      }
    if ((mbits & ((1u << m) - 1u)) == 0u) {
      // mask-free interior: the elimination coefficients come from the tables
      T dt = 0;
#pragma unroll
      for (int e = 0; e < LMAX - 1; ++e)
        if (e < m) {
          dt = (dd[e] - TAB(4, e) * dt) * TAB(0, e);
          dd[e] = dt;
        }
      T dh = 0;
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
      T at = 0, ct = 0, dt = 0;
#pragma unroll
      for (int e = 0; e < LMAX - 1; ++e)
        if (e < m) {
          const int i = lo + e;
          const int64_t o = base + (int64_t)i * es;
          T a, b, c;
          row_coef(K, i, a, b, c);
          if ((mbits >> e) & 1u) {
            a = 0;
            b = 1;
            c = 0;
          }
          const T inv = T(1) / (b - a * ct);
          at = (e == 0) ? a * inv : -a * at * inv;
          ct = c * inv;
          dt = (dd[e] - a * dt) * inv;
          dd[e] = dt;
          K.sa[o] = at;
          K.sc[o] = ct;
        }
      T ah = 0, ch = 0, dh = 0;
#pragma unroll
      for (int e = LMAX - 2; e >= 0; --e)
        if (e < m) {
          const int64_t o = base + (int64_t)(lo + e) * es;
          const T at_e = K.sa[o], ct_e = K.sc[o];
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
      az = 0;
      bz = 1;
      cz = 0;
    }
  }
  // LDS: 8 arrays of P doubles per line; neighbouring lanes (consecutive
  // lines in the z/y sweeps, consecutive segments in the x sweep) take
  // consecutive words
  if (MODE == 0) __syncthreads();  // the row buffer becomes the separator arrays
  const int TL = K.tl;
  const bool rowmajor = (MODE == 0);
  auto at = [&](int f, int seg) -> T& {
    return rowmajor ? sm[((size_t)f * TL + lb) * P + seg] : sm[((size_t)f * P + seg) * TL + lb];
  };
  if (active) {
    at(0, s) = a0;
    at(1, s) = c0;
    at(2, s) = valid ? dd[0] : T(0);
  }
  __syncthreads();
  T ra = 0, rb = 1, rg = 0, rd = 0;  // this segment's separator row
  if (active) {
    int sn = s + 1;
    T czz = cz;
    if (sn == P) {
      sn = 0;
      if (!K.cyc) czz = 0;
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
      T na = 0, nb = 1, ng = 0, nd = 0;
      if (active) {
        int im = s - st, ip = s + st;
        T am = 0, bm = 1, gm = 0, dm = 0, ap = 0, bp = 1, gp = 0, dp = 0;
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
        const T k1 = ra / bm, k2 = rg / bp;
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
    if (active && s == 0) reduced_solve_cyclic<T>(at, P);
  }
  __syncthreads();
  if (valid) {
    const T zr = at(7, s);
    const T zl = (s > 0) ? at(7, s - 1) : (K.cyc ? at(7, P - 1) : T(0));
    const bool fast = (mbits & ((1u << m) - 1u)) == 0u;
#pragma unroll
    for (int e = 0; e < LMAX; ++e)
      if (e < len) {
        const int64_t o = base + (int64_t)(lo + e) * es;
        T x = zr;
        if (e < m) x = fast ? dd[e] - TAB(2, e) * zl - TAB(3, e) * zr
                            : dd[e] - K.sa[o] * zl - K.sc[o] * zr;
        if (MODE == 0) {
          if (e < m) dd[e] = x; else dz = x;
        } else if (MODE == 2) {
          K.u[o] = uu[MODE == 2 ? e : 0] + (double)x;
        } else {
          K.d[o] = x;
        }
      }
  }
  if (MODE == 0) {
    __syncthreads();  // every thread has read the separator values
    if (valid) {
#pragma unroll
      for (int e = 0; e < LMAX; ++e)
        if (e < len) rowbuf[xpos(e)] = (e < m) ? dd[e] : dz;
    }
    __syncthreads();
    T* xdst = K.d + (xsrc - K.d);
    for (int e = tid; e < xrows * K.n; e += blockDim.x) {
      const int r = e / K.n, c = e - r * K.n;
      xdst[e] = rowbuf[r * RS + c + (c >> 4)];
    }
  }
}

// 16 bytes of T as a native vector (kept in registers where an array of them
// lives across a loop)
template <typename T> struct Vec16;
template <> struct Vec16<double> { using type = double __attribute__((ext_vector_type(2))); };
template <> struct Vec16<float> { using type = float __attribute__((ext_vector_type(4))); };

// a group's rows and this lane's mask word for the x sweep below (a segment
// starts at a multiple of 16: its bits lie in one word)
template <typename T, int VPL>
__device__ __forceinline__ void xw_fetch(const LineK<T>& K, typename Vec16<T>::type (&pf)[VPL],
                                         uint32_t& pmw, int64_t gg, int RW, int64_t nl,
                                         int64_t e0, int lane, int rr, int s) {
  using V = typename Vec16<T>::type;
  constexpr int VN = 16 / sizeof(T);
  const int n = K.n;
  const int64_t g0 = e0 + gg * RW * n;
  const int64_t nv = (nl - gg * RW) * n / VN;  // vectors left in the sweep
#pragma unroll
  for (int v = 0; v < VPL; ++v) {
    // (past the end: a repeat of the last vector, so that the loop keeps a
    // fixed trip count and the array stays in registers)
    const int q = lane + 64 * v < nv ? lane + 64 * v : (int)nv - 1;
    pf[v] = *reinterpret_cast<const V*>(K.d + g0 + (int64_t)q * VN);
  }
  if (gg * RW + rr < nl) pmw = K.mask[(g0 + (int64_t)rr * n + s * LMAX) >> 5];
}

// x sweep with one wavefront per group of 64/P rows, for lines of n = P*LMAX
// rows with P a power of two (4 <= P <= 64): lane rr*P + s holds segment s of
// row rr.  The group's rows are staged through the wavefront's own LDS region
// (16-byte loads and stores, a 16-byte pad after every segment so that the
// lanes' segment reads fall on distinct banks), and the separator system is
// solved by cyclic reduction over cross-lane reads, so the wavefronts of a
// block never wait for each other.  Equal segments of a constant-coefficient
// line share one set of elimination tables (segment 0's).
//
// A group always holds 64 LMAX values (64/P rows of P LMAX).  The grid holds
// only as many wavefronts as are resident at once; each takes the groups
// g, g + W, g + 2W, ... (W wavefronts in all) and loads the next group's rows
// and mask words into registers before it solves the current one, so that
// the chip's loads stay in flight through the elimination and the stores
// instead of arriving in one wave of requests per round of blocks.
template <typename T, bool G = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_line_xw(GArg<LineK<T>, G> grp_arg_) {
  uint3 bid, gdim;
  const LineK<T>& K = grp_enter<LineK<T>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  using V = typename Vec16<T>::type;
  constexpr int VN = 16 / sizeof(T);  // values per 16 bytes
  constexpr int SEGS = LMAX + VN;     // padded segment
  constexpr int GV = 64 * LMAX / VN;  // 16-byte vectors per group
  constexpr int VPL = GV / 64;        // ... per lane
  extern __shared__ __align__(16) unsigned char ldsraw[];
  T* lds = reinterpret_cast<T*>(ldsraw);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int P = K.P, n = K.n;
  const int RW = 64 / P;             // rows per group
  const int RS = (n / LMAX) * SEGS;  // padded row
  T* tab = lds;                      // [LINE_NTAB][LMAX]
  T* rows = lds + LINE_NTAB * LMAX + (size_t)wv * RW * RS;
  for (int q = threadIdx.x; q < LINE_NTAB * LMAX; q += blockDim.x)
    tab[q] = K.tab[(size_t)(q / LMAX) * P * LINE_TLD + q % LMAX];
  __syncthreads();
  const int64_t nl = (int64_t)K.nj * K.nz;  // rows of the sweep
  const int64_t ng = (nl + RW - 1) / RW;    // groups
  const int64_t gstep = (int64_t)gdim.x * (blockDim.x >> 6);
  int64_t g = (int64_t)bid.x * (blockDim.x >> 6) + wv;
  if (g >= ng) return;  // the whole wavefront is past the end
  const int lgn = 31 - __clz(n);  // n = P LMAX is a power of two
  const int rr = lane / P, s = lane % P;
  const int grp = rr * P;  // first lane of this row
  T* seg = rows + rr * RS + s * SEGS;
  const int m = LMAX - 1;  // interior rows; row m is the separator
  const int nxt = grp + ((s + 1) & (P - 1)), prv = grp + ((s - 1) & (P - 1));
  const int64_t e0 = (int64_t)K.j0 * K.nz * n;  // first element of the sweep
  // a group's rows and this lane's mask word (a segment starts at a multiple
  // of 16: its bits lie in one word); vectors past the sweep are not loaded
  V pf[VPL];
  uint32_t pmw = 0;
  xw_fetch<T, VPL>(K, pf, pmw, g, RW, nl, e0, lane, rr, s);
  for (; g < ng; g += gstep) {
    const int64_t r0 = g * RW;
    const int nrow = (int)((r0 + RW <= nl) ? RW : nl - r0);
    const int64_t g0 = e0 + r0 * n;  // first element of the group
    const int nv = nrow * n / VN;
    const bool valid = rr < nrow;
    const int64_t base = g0 + (int64_t)rr * n + s * LMAX;  // first element of the segment
    // stage the group's rows: value c of row r at rows[r*RS + (c/LMAX)*SEGS + c%LMAX]
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
      // rows past the group's end (a ragged last group) take unused values:
      // they stay inside this wavefront's region
      const int q = lane + 64 * v;
      const int c0 = q * VN, r = c0 >> lgn, c = c0 & (n - 1);
      *reinterpret_cast<V*>(rows + r * RS + (c / LMAX) * SEGS + c % LMAX) = pf[v];
    }
    const uint32_t mbits = valid ? (pmw >> (uint32_t)(base & 31)) & ((1u << LMAX) - 1u) : 0u;
    wave_sync();
    if (g + gstep < ng) xw_fetch<T, VPL>(K, pf, pmw, g + gstep, RW, nl, e0, lane, rr, s);
    T dd[LMAX];
    T dz = 0, az = 0, bz = 1, cz = 0;
    T a0 = 0, c0 = 0, ahl = 0, chl = 0, dhl = 0;
    if (valid) {
#pragma unroll
      for (int e = 0; e < LMAX; ++e) dd[e] = seg[e];
#pragma unroll
      for (int e = 0; e < LMAX; ++e)
        if ((mbits >> e) & 1u) dd[e] = T(0);
      dz = dd[m];
      if ((mbits & ((1u << m) - 1u)) == 0u) {
        T dt = 0;
#pragma unroll
        for (int e = 0; e < m; ++e) {
          dt = (dd[e] - tab[4 * LMAX + e] * dt) * tab[e];
          dd[e] = dt;
        }
        T dh = dd[m - 1];
        dhl = dh;
#pragma unroll
        for (int e = m - 2; e >= 0; --e) {
          dh = dd[e] - tab[LMAX + e] * dh;
          dd[e] = dh;
        }
        a0 = tab[2 * LMAX];
        c0 = tab[3 * LMAX];
        ahl = tab[2 * LMAX + m - 1];
        chl = tab[3 * LMAX + m - 1];
      } else {
        // identity rows inside the segment: coefficients through the scratch
        T at = 0, ct = 0, dt = 0;
#pragma unroll
        for (int e = 0; e < m; ++e) {
          T a = K.a, b = K.b, c = K.c;
          if ((mbits >> e) & 1u) {
            a = 0;
            b = 1;
            c = 0;
          }
          const T inv = T(1) / (b - a * ct);
          at = (e == 0) ? a * inv : -a * at * inv;
          ct = c * inv;
          dt = (dd[e] - a * dt) * inv;
          dd[e] = dt;
          K.sa[base + e] = at;
          K.sc[base + e] = ct;
        }
        T ah = 0, ch = 0, dh = 0;
#pragma unroll
        for (int e = m - 1; e >= 0; --e) {
          const T at_e = K.sa[base + e], ct_e = K.sc[base + e];
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
          K.sa[base + e] = ah;
          K.sc[base + e] = ch;
        }
        a0 = ah;
        c0 = ch;
      }
      az = K.a;
      bz = K.b;
      cz = K.c;
      if ((mbits >> m) & 1u) {
        az = 0;
        bz = 1;
        cz = 0;
      }
    }
    // separator row of this segment (every lane takes part in the cross-lane
    // reads; lanes past the group's rows carry identity rows)
    const T a0n = lane_read(a0, nxt), c0n = lane_read(c0, nxt);
    const T d0n = lane_read(valid ? dd[0] : T(0), nxt);
    T ra = -az * ahl;
    T rb = bz - az * chl - cz * a0n;
    T rg = -cz * c0n;
    T rd = dz - az * dhl - cz * d0n;
    // cyclic reduction: a cyclic system of 2^k rows closes with couplings onto
    // the row itself
    for (int st = 1; st < P; st <<= 1) {
      const int im = grp + ((s - st) & (P - 1)), ip = grp + ((s + st) & (P - 1));
      const T am = lane_read(ra, im), bm = lane_read(rb, im), gm = lane_read(rg, im),
              dm = lane_read(rd, im);
      const T ap = lane_read(ra, ip), bp = lane_read(rb, ip), gp = lane_read(rg, ip),
              dp = lane_read(rd, ip);
      const T k1 = ra / bm, k2 = rg / bp;
      const T na = -am * k1, ng_ = -gp * k2;
      rb = rb - gm * k1 - ap * k2;
      rd = rd - dm * k1 - dp * k2;
      ra = na;
      rg = ng_;
    }
    const T zr = rd / (ra + rb + rg);
    const T zl = lane_read(zr, prv);
    if (valid) {
      const bool fast = (mbits & ((1u << m) - 1u)) == 0u;
#pragma unroll
      for (int e = 0; e < m; ++e)
        seg[e] = fast ? dd[e] - tab[2 * LMAX + e] * zl - tab[3 * LMAX + e] * zr
                      : dd[e] - K.sa[base + e] * zl - K.sc[base + e] * zr;
      seg[m] = zr;
    }
    wave_sync();
#pragma unroll
    for (int v = 0; v < VPL; ++v) {
      // past the group's end: the last vector again (the same value)
      const int q = lane + 64 * v < nv ? lane + 64 * v : nv - 1;
      const int c0_ = q * VN, r = c0_ >> lgn, c = c0_ & (n - 1);
      *reinterpret_cast<V*>(K.d + g0 + c0_) =
          *reinterpret_cast<const V*>(rows + r * RS + (c / LMAX) * SEGS + c % LMAX);
    }
    wave_sync();  // the rows are read out before the next group is staged
  }
}

// z and y sweeps for lines of n = P*LMAX rows (every segment LMAX rows) on
// grids with nx a multiple of 16.  A block takes 16 lines of consecutive x
// (a wavefront's loads then cover 128-byte row pieces).
//  1. thread (line lb, segment s) loads its segment (and, for y, the velocity
//     it adds to), takes the forcing-mask bits of its rows from one word per
//     row that the 16 lanes of the segment load together, and eliminates the
//     interior rows;
//  2. the separator rows are formed in LDS and re-read transposed: a line's
//     PP (P rounded up to a power of two) separators then sit in consecutive
//     lanes of one wavefront, which solves them by cyclic reduction over
//     cross-lane reads (rows past P act as identity rows);
//  3. each thread reconstructs and stores its rows.
// Four block barriers in all.
// coefficients of row i: per-row arrays for the y sweep, the constants otherwise
template <int MODE, typename T>
__device__ __forceinline__ void col_coef(const LineK<T>& K, int i, T& a, T& b, T& c) {
  if (MODE == 2) {
    a = K.A[i];
    b = K.B[i];
    c = K.C[i];
  } else {
    a = K.a;
    b = K.b;
    c = K.c;
  }
}

// Register form of the column sweep for the wall-normal lines of 12- and
// 16-row segments: every row of a segment is addressed and held in
// registers through the whole launch, the rare segments with identity rows
// included (their coefficients through the scratch).  Where lines cross a
// body often (a plate spanning the wall-normal lines) it is faster than the
// form below, whose rare path goes through memory.
template <typename T, int MODE, int SL, int TL, bool G = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(SL == 12 ? 5 : 1)))
void k_line_col_reg(GArg<LineK<T>, G> grp_arg_) {
  uint3 bid, gdim;
  const LineK<T>& K = grp_enter<LineK<T>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  // TL lines per block: 16, or 32 in FP32 (a wavefront's loads then cover
  // 128-byte row pieces in both), and 32 with the long segments (24 or 32
  // rows) of the large planes
  constexpr int SP = TL + 1;   // padded stride of the separator arrays
  extern __shared__ __align__(16) unsigned char ldsraw[];
  T* lds = reinterpret_cast<T*>(ldsraw);
  const int tid = threadIdx.x;
  const int P = K.P, PP = K.PP;
  const int tP = K.tab1 ? 1 : P;
  T* tabs = lds;                             // [LINE_NTAB][SL][tP]
  T* Y = tabs + LINE_NTAB * SL * tP;         // a0, c0, d0 of each segment; then z
  T* X = Y + 3 * PP * SP;                    // separator rows ra, rb, rg, rd
  uint32_t* mws = reinterpret_cast<uint32_t*>(X + 4 * PP * SP);  // [P][SL] mask words
  for (int q = tid; q < LINE_NTAB * tP * SL; q += blockDim.x) {
    const int qe = q / tP, ss = q % tP, qq = qe / SL, ee = qe % SL;
    tabs[q] = K.tab[((size_t)qq * P + ss) * LINE_TLD + ee];  // global: LINE_TLD per segment
  }
  const int lb = tid % TL, s = tid / TL;
  const bool active = s < P;
  // large planes: whole z rows (y sweep) or y planes (z sweep) per XCD, all
  // x tiles of a row together, in a 1-D grid (as in the lean kernel below);
  // small planes: z-major 2-D grid (consecutive blocks on different z rows,
  // hence different memory channels), x-tile fastest for the z sweep
  int bx, by;
  if (K.xrow) {
    const int nxt = K.nx / TL;
    const int nout = (MODE == 2) ? K.nz : K.nj;
    const int64_t b = bid.x;
    const int64_t r = b / NUM_XCD;
    by = (int)(r / nxt) * NUM_XCD + (int)(b % NUM_XCD);
    bx = (int)(r % nxt);
    if (by >= nout) return;  // padding of the last round
  } else {
    bx = (MODE == 2) ? (int)bid.y : (int)bid.x;
    by = (MODE == 2) ? (int)bid.x : (int)bid.y;
  }
  const int i0 = bx * TL;
  const int ts = K.tab1 ? 0 : s;
#define CTAB(q, e) tabs[((q) * SL + (e)) * tP + ts]
  // element (row r of line lb): blk[lb + r * es]
  const int64_t es = (MODE == 1) ? K.nx : K.plane;
  const int64_t boff = (MODE == 1) ? (int64_t)(K.j0 + by) * K.plane + i0
                                   : (int64_t)K.j0 * K.plane + (int64_t)by * K.nx + i0;
  const int lo = s * SL;
  constexpr int m = SL - 1;
  T dd[SL];
  double uu[MODE == 2 ? SL : 1];
  T dz = 0, az = 0, bz = 1, cz = 0;
  T a0 = 0, c0 = 0, ahl = 0, chl = 0, dhl = 0;
  uint32_t mbits = 0;
  // rows are addressed from the wavefront's first row (a uniform base) plus
  // a 32-bit byte offset, one register per row instead of a 64-bit address
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t wrow = (int64_t)wv * (64 / TL) * SL;  // first row of the wavefront
  const T* dbase = K.d + boff + wrow * es;
  const double* ubase = (MODE == 2) ? K.u + boff + wrow * es : nullptr;
  const uint32_t lrow = (uint32_t)(lo - wrow);           // this segment's first row, from wrow
  auto boffs = [&](int e, uint32_t sz) -> uint32_t {
    return ((uint32_t)lb + (lrow + (uint32_t)e) * (uint32_t)es) * sz;
  };
  if (active) {
#pragma unroll
    for (int e = 0; e < SL; ++e)
      dd[e] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(dbase) + boffs(e, sizeof(T)));
    // lane lb < SL fetches the mask word of row lo + lb (bits i0 .. i0+TL-1
    // of the row: within one word, nx and i0 being multiples of TL)
    static_assert(SL <= TL, "one mask word per lane");
    if (lb < SL) {
      const int64_t rb = (MODE == 1) ? ((int64_t)(K.j0 + by) * K.nz + lo + lb) * K.nx
                                     : ((int64_t)(K.j0 + lo + lb) * K.nz + by) * K.nx;
      const int64_t bit = rb + i0;
      const uint32_t w = K.mask[bit >> 5] >> (uint32_t)(bit & 31);
      mws[s * SL + lb] = (TL == 32) ? w : (w & ((1u << (TL & 31)) - 1u));
    }
  }
  __syncthreads();  // tables and mask words
  if (active) {
#pragma unroll
    for (int e = 0; e < SL; ++e) mbits |= ((mws[s * SL + e] >> lb) & 1u) << e;
#pragma unroll
    for (int e = 0; e < SL; ++e)
      if ((mbits >> e) & 1u) dd[e] = T(0);
    dz = dd[m];
    if ((mbits & ((1u << m) - 1u)) == 0u) {
      T dt = 0;
#pragma unroll
      for (int e = 0; e < m; ++e) {
        dt = (dd[e] - CTAB(4, e) * dt) * CTAB(0, e);
        dd[e] = dt;
      }
      T dh = dd[m - 1];
      dhl = dh;
#pragma unroll
      for (int e = m - 2; e >= 0; --e) {
        dh = dd[e] - CTAB(1, e) * dh;
        dd[e] = dh;
      }
      a0 = CTAB(2, 0);
      c0 = CTAB(3, 0);
      ahl = CTAB(2, m - 1);
      chl = CTAB(3, m - 1);
    } else {
      // identity rows inside the segment: coefficients through the scratch
      T at = 0, ct = 0, dt = 0;
      for (int e = 0; e < m; ++e) {
        const int64_t o = boff + lb + (lo + e) * es;
        T a, b, c;
        col_coef<MODE>(K, lo + e, a, b, c);
        if ((mbits >> e) & 1u) {
          a = 0;
          b = 1;
          c = 0;
        }
        const T inv = T(1) / (b - a * ct);
        at = (e == 0) ? a * inv : -a * at * inv;
        ct = c * inv;
        dt = (dd[e] - a * dt) * inv;
        dd[e] = dt;
        K.sa[o] = at;
        K.sc[o] = ct;
      }
      T ah = 0, ch = 0, dh = 0;
      for (int e = m - 1; e >= 0; --e) {
        const int64_t o = boff + lb + (lo + e) * es;
        const T at_e = K.sa[o], ct_e = K.sc[o];
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
    col_coef<MODE>(K, lo + m, az, bz, cz);
    if ((mbits >> m) & 1u) {
      az = 0;
      bz = 1;
      cz = 0;
    }
    Y[(0 * PP + s) * SP + lb] = a0;
    Y[(1 * PP + s) * SP + lb] = c0;
    Y[(2 * PP + s) * SP + lb] = dd[0];
  }
  __syncthreads();  // a0, c0, d0 of every segment
  if (active) {
    int sn = s + 1;
    T czz = cz;
    if (sn == P) {
      sn = 0;
      if (!K.cyc) czz = 0;
    }
    X[(0 * PP + s) * SP + lb] = -az * ahl;
    X[(1 * PP + s) * SP + lb] = bz - az * chl - czz * Y[(0 * PP + sn) * SP + lb];
    X[(2 * PP + s) * SP + lb] = -czz * Y[(1 * PP + sn) * SP + lb];
    X[(3 * PP + s) * SP + lb] = dz - az * dhl - czz * Y[(2 * PP + sn) * SP + lb];
  }
  __syncthreads();  // separator rows
  // transposed: thread (line lt, separator st) in PP consecutive lanes
  {
    const int lt = tid / PP, st = tid % PP;
    const int lane = tid & 63, grp = lane - st;
    T ra = 0, rb = 1, rg = 0, rd = 0;
    if (lt < TL && st < P) {
      ra = X[(0 * PP + st) * SP + lt];
      rb = X[(1 * PP + st) * SP + lt];
      rg = X[(2 * PP + st) * SP + lt];
      rd = X[(3 * PP + st) * SP + lt];
    }
    for (int step = 1; step < PP; step <<= 1) {
      int im = st - step, ip = st + step;
      bool hm = true, hp = true;
      if (K.cyc) {
        im &= PP - 1;
        ip &= PP - 1;
      } else {
        hm = im >= 0;
        hp = ip < PP;
      }
      const int sm_ = grp + (hm ? im : st), sp_ = grp + (hp ? ip : st);
      T am = lane_read(ra, sm_), bm = lane_read(rb, sm_), gm = lane_read(rg, sm_),
        dm = lane_read(rd, sm_);
      T ap = lane_read(ra, sp_), bp = lane_read(rb, sp_), gp = lane_read(rg, sp_),
        dp = lane_read(rd, sp_);
      if (!hm) {
        am = 0;
        bm = 1;
        gm = 0;
        dm = 0;
      }
      if (!hp) {
        ap = 0;
        bp = 1;
        gp = 0;
        dp = 0;
      }
      const T k1 = ra / bm, k2 = rg / bp;
      const T na = -am * k1, ng = -gp * k2;
      rb = rb - gm * k1 - ap * k2;
      rd = rd - dm * k1 - dp * k2;
      ra = na;
      rg = ng;
    }
    if (lt < TL && st < P) Y[st * SP + lt] = K.cyc ? rd / (ra + rb + rg) : rd / rb;
  }
  if (MODE == 2 && active) {
    // the velocity the solution is added to: loaded here, where the
    // registers of the separator solve are free, in flight over the barrier
#pragma unroll
    for (int e = 0; e < SL; ++e)
      uu[e] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(ubase) + boffs(e, 8));
  }
  __syncthreads();  // separator values
  if (active) {
    const T zr = Y[s * SP + lb];
    const T zl = (s > 0) ? Y[(s - 1) * SP + lb] : (K.cyc ? Y[(P - 1) * SP + lb] : T(0));
    if ((mbits & ((1u << m) - 1u)) == 0u) {
#pragma unroll
      for (int e = 0; e < m; ++e) dd[e] = dd[e] - CTAB(2, e) * zl - CTAB(3, e) * zr;
    } else {
#pragma unroll
      for (int e = 0; e < m; ++e) {
        const int64_t o = boff + lb + (lo + e) * es;
        dd[e] = dd[e] - K.sa[o] * zl - K.sc[o] * zr;
      }
    }
    dd[m] = zr;
#pragma unroll
    for (int e = 0; e < SL; ++e) {
      if (MODE == 2)
        *reinterpret_cast<double*>(reinterpret_cast<char*>(const_cast<double*>(ubase)) + boffs(e, 8)) =
            uu[MODE == 2 ? e : 0] + (double)dd[e];
      else
        *reinterpret_cast<T*>(reinterpret_cast<char*>(const_cast<T*>(dbase)) + boffs(e, sizeof(T))) =
            dd[e];
    }
#undef CTAB
  }
}


// Lean form of the column sweep (z sweeps, whose lines seldom meet a body,
// and the 24- and 32-row segments of the large planes): rows through buffer
// descriptors, and segments with identity rows through memory, so that the
// common path keeps few registers (two blocks of 1024 threads per CU for
// the 32-row FP32 z sweep).
template <typename T, int MODE, int SL, int TL, bool G = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(SL == 12 ? 5 : ((SL == 32 || SL == 24) ? 8 : 1))))
void k_line_col(GArg<LineK<T>, G> grp_arg_) {
  uint3 bid, gdim;
  const LineK<T>& K = grp_enter<LineK<T>, G>(grp_arg_, bid, gdim);
  (void)bid;
  (void)gdim;
  // TL lines per block: 16, or 32 in FP32 (a wavefront's loads then cover
  // 128-byte row pieces in both), and 32 with the long segments (24 or 32
  // rows) of the large planes
  constexpr int SP = TL + 1;   // padded stride of the separator arrays
  extern __shared__ __align__(16) unsigned char ldsraw[];
  T* lds = reinterpret_cast<T*>(ldsraw);
  const int tid = threadIdx.x;
  const int P = K.P, PP = K.PP;
  const int tP = K.tab1 ? 1 : P;
  T* tabs = lds;                             // [LINE_NTAB][SL][tP]
  T* Y = tabs + LINE_NTAB * SL * tP;         // a0, c0, d0 of each segment; then z
  T* X = Y + 3 * PP * SP;                    // separator rows ra, rb, rg, rd
  uint32_t* mws = reinterpret_cast<uint32_t*>(X + 4 * PP * SP);  // [P][SL] mask words
  // y sweep: the rows' coefficients a, b, c (read by segments with identity
  // rows), after the mask words
  T* cf = reinterpret_cast<T*>(mws + P * SL);
  for (int q = tid; q < LINE_NTAB * tP * SL; q += blockDim.x) {
    const int qe = q / tP, ss = q % tP, qq = qe / SL, ee = qe % SL;
    tabs[q] = K.tab[((size_t)qq * P + ss) * LINE_TLD + ee];  // global: LINE_TLD per segment
  }
  if (MODE == 2) {
    const int nl = P * SL;
    for (int q = tid; q < 3 * nl; q += blockDim.x)
      cf[q] = (q < nl) ? K.A[q] : (q < 2 * nl ? K.B[q - nl] : K.C[q - 2 * nl]);
  }
  const int lb = tid % TL, s = tid / TL;
  const bool active = s < P;
  // y sweep: a 1-D grid in which each XCD (blocks
  // are dealt to the 8 XCDs round robin) takes whole z rows, one after the
  // other, all x tiles of a row together: every row of a line lies in its
  // own page, and the blocks of one z row then share the address
  // translation of each of those pages in their XCD's L2 TLB (z-major blocks
  // met each page once per x tile, a page-table read each time)
  // The z sweep likewise: each XCD takes whole y planes, all x tiles of a
  // plane together (the rows of a z line are a plane's z rows).
  int bx, by;
  {
    const int nxt = K.nx / TL;
    const int nout = (MODE == 2) ? K.nz : K.nj;  // z rows (y sweep) or planes (z sweep)
    const int64_t b = bid.x;
    const int64_t r = b / NUM_XCD;
    by = (int)(r / nxt) * NUM_XCD + (int)(b % NUM_XCD);
    bx = (int)(r % nxt);
    if (by >= nout) return;  // padding of the last round
  }
  const int i0 = bx * TL;
  const int ts = K.tab1 ? 0 : s;
#define CTAB(q, e) tabs[((q) * SL + (e)) * tP + ts]
  // element (row r of line lb): blk[lb + r * es]
  const int64_t es = (MODE == 1) ? K.nx : K.plane;
  const int64_t boff = (MODE == 1) ? (int64_t)(K.j0 + by) * K.plane + i0
                                   : (int64_t)K.j0 * K.plane + (int64_t)by * K.nx + i0;
  const int lo = s * SL;
  constexpr int m = SL - 1;
  T dd[SL];
  // y sweep: the velocity of the first NPRE rows is prefetched over the last
  // barrier, the rest is read at the store
  constexpr int NPRE = (MODE == 2) ? (SL >= 24 ? SL / 2 : SL) : 0;
  constexpr bool UPRE = NPRE > 0;
  constexpr int RC = 4;  // rows per memory round trip on the rare path
  double uu[UPRE ? NPRE : 1];
  T dz = 0, az = 0, bz = 1, cz = 0;
  T a0 = 0, c0 = 0, d0 = 0, ahl = 0, chl = 0, dhl = 0;
  // forcing rows: any among the segment's interior rows (then the rare
  // path), and the separator row
  bool rare = false, last_forced = false;
  // rows are addressed through buffer descriptors based at the wavefront's
  // first row: one per-lane byte offset (line and segment) and a uniform
  // row offset in a scalar register, instead of one address per row held
  // from the loads to the stores
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int WROWS = (64 / TL) * SL;                   // rows of one wavefront
  const int64_t wrow = (int64_t)wv * WROWS;               // its first row
  const uint32_t lrow = (uint32_t)(lo - wrow);            // this segment's first row, from wrow
  const __amdgpu_buffer_rsrc_t dres =
      buf_rsrc(K.d + boff + wrow * es, (uint32_t)(WROWS * es * (int64_t)sizeof(T)));
  const __amdgpu_buffer_rsrc_t ures =
      buf_rsrc((MODE == 2) ? K.u + boff + wrow * es : nullptr, (uint32_t)(WROWS * es * 8));
  const uint32_t vline = (uint32_t)lb + lrow * (uint32_t)es;  // element offset of row 0
  const uint32_t rstride = (uint32_t)es;                      // elements per row
  // the line-solve scratch (coefficients of segments with identity rows)
  // has the layout of d
  const __amdgpu_buffer_rsrc_t sares =
      buf_rsrc(K.sa + boff + wrow * es, (uint32_t)(WROWS * es * (int64_t)sizeof(T)));
  const __amdgpu_buffer_rsrc_t scres =
      buf_rsrc(K.sc + boff + wrow * es, (uint32_t)(WROWS * es * (int64_t)sizeof(T)));
  auto roff = [&](int e) -> uint32_t { return (uint32_t)e * rstride * (uint32_t)sizeof(T); };
  const uint32_t vlb = vline * (uint32_t)sizeof(T);
  auto u_at = [&](int e) -> double {
    return (e < NPRE) ? uu[e < NPRE ? e : 0] : buf_ld<double>(ures, vline * 8u, (uint32_t)e * rstride * 8u);
  };
  uint32_t mw = 0;  // lanes lb < SL: the mask word of row lo + lb
  if (active) {
#pragma unroll
    for (int e = 0; e < SL; ++e)
      dd[e] = buf_ld<T>(dres, vlb, roff(e));
    // lane lb < SL fetches the mask word of row lo + lb (bits i0 .. i0+TL-1
    // of the row: within one word, nx and i0 being multiples of TL)
    static_assert(SL <= TL, "one mask word per lane");
    if (lb < SL) {
      const int64_t rb = (MODE == 1) ? ((int64_t)(K.j0 + by) * K.nz + lo + lb) * K.nx
                                     : ((int64_t)(K.j0 + lo + lb) * K.nz + by) * K.nx;
      const int64_t bit = rb + i0;
      const uint32_t w = K.mask[bit >> 5] >> (uint32_t)(bit & 31);
      mw = (TL == 32) ? w : (w & ((1u << (TL & 31)) - 1u));
      mws[s * SL + lb] = mw;
    }
  }
  {
    // the OR of the interior rows' words over the segment's TL lanes (all
    // lanes take part; inactive ones hold 0) and the separator row's word
    uint32_t wi = (lb < m) ? mw : 0u;
#pragma unroll
    for (int o = 1; o < TL; o <<= 1) wi |= (uint32_t)__shfl_xor((int)wi, o, TL);
    const uint32_t wl = (uint32_t)__shfl((int)mw, m, TL);
    rare = (wi >> lb) & 1u;
    last_forced = (wl >> lb) & 1u;
  }
  __syncthreads();  // tables and mask words
  if (active) {
    // a forcing row's value is 0 (its update is zero); the interior rows of a
    // segment that holds one take the rare path below, which applies it
    dz = last_forced ? T(0) : dd[m];
    if (!rare) {
      T dt = 0;
#pragma unroll
      for (int e = 0; e < m; ++e) {
        dt = (dd[e] - CTAB(4, e) * dt) * CTAB(0, e);
        dd[e] = dt;
      }
      T dh = dd[m - 1];
      dhl = dh;
#pragma unroll
      for (int e = m - 2; e >= 0; --e) {
        dh = dd[e] - CTAB(1, e) * dh;
        dd[e] = dh;
      }
      a0 = CTAB(2, 0);
      c0 = CTAB(3, 0);
      d0 = dd[0];
      ahl = CTAB(2, m - 1);
      chl = CTAB(3, m - 1);
    } else {
      // identity rows inside the segment (rare): the eliminated rows and
      // their coefficients go through memory (the rows in place in d, the
      // coefficients in the scratch).  This path defines no row value in
      // registers: a divergent branch runs both sides, so values of its own
      // would need registers beside the common path's rows (twice the
      // registers, half the occupancy).  It reads the loaded rows in dd, and
      // fetches its operands RC rows at a time, so that it waits on memory
      // once per RC rows with few registers in flight.
      T at = 0, ct = 0, dt = 0;
#pragma unroll
      for (int e = 0; e < m; ++e) {
        if (e > 0 && e % RC == 0) __builtin_amdgcn_sched_barrier(0);
        T a, b, c;
        if (MODE == 2) {
          a = cf[lo + e];
          b = cf[P * SL + lo + e];
          c = cf[2 * P * SL + lo + e];
        } else {
          col_coef<MODE>(K, lo + e, a, b, c);
        }
        const bool msk = (mws[s * SL + e] >> lb) & 1u;
        if (msk) {
          a = 0;
          b = 1;
          c = 0;
        }
        const T inv = T(1) / (b - a * ct);
        at = (e == 0) ? a * inv : -a * at * inv;
        ct = c * inv;
        dt = ((msk ? T(0) : dd[e]) - a * dt) * inv;
        if (e < m - 1) {
          buf_st(dt, dres, vlb, roff(e));
          buf_st(at, sares, vlb, roff(e));
          buf_st(ct, scres, vlb, roff(e));
        }
      }
      // back substitution from row m - 1 (its values still in registers)
      T ah = at, ch = ct, dh = dt;
      ahl = ah;
      chl = ch;
      dhl = dh;
      buf_st(dh, dres, vlb, roff(m - 1));
      buf_st(ah, sares, vlb, roff(m - 1));
      buf_st(ch, scres, vlb, roff(m - 1));
#pragma unroll
      for (int e1 = m - 2; e1 >= 0; e1 -= RC) {
        __builtin_amdgcn_sched_barrier(0);
        T ca[RC], cc[RC], cd[RC];
#pragma unroll
        for (int q = 0; q < RC; ++q)
          if (e1 - q >= 0) {
            ca[q] = buf_ld<T>(sares, vlb, roff(e1 - q));
            cc[q] = buf_ld<T>(scres, vlb, roff(e1 - q));
            cd[q] = buf_ld<T>(dres, vlb, roff(e1 - q));
          }
#pragma unroll
        for (int q = 0; q < RC; ++q)
          if (e1 - q >= 0) {
            dh = cd[q] - cc[q] * dh;
            ah = ca[q] - cc[q] * ah;
            ch = -cc[q] * ch;
            buf_st(dh, dres, vlb, roff(e1 - q));
            buf_st(ah, sares, vlb, roff(e1 - q));
            buf_st(ch, scres, vlb, roff(e1 - q));
          }
      }
      __builtin_amdgcn_sched_barrier(0);
      a0 = ah;
      c0 = ch;
      d0 = dh;  // dd[] stays as loaded (unused on this path)
    }
    col_coef<MODE>(K, lo + m, az, bz, cz);
    if (last_forced) {
      az = 0;
      bz = 1;
      cz = 0;
    }
    Y[(0 * PP + s) * SP + lb] = a0;
    Y[(1 * PP + s) * SP + lb] = c0;
    Y[(2 * PP + s) * SP + lb] = d0;
  }
  __syncthreads();  // a0, c0, d0 of every segment
  if (active) {
    int sn = s + 1;
    T czz = cz;
    if (sn == P) {
      sn = 0;
      if (!K.cyc) czz = 0;
    }
    X[(0 * PP + s) * SP + lb] = -az * ahl;
    X[(1 * PP + s) * SP + lb] = bz - az * chl - czz * Y[(0 * PP + sn) * SP + lb];
    X[(2 * PP + s) * SP + lb] = -czz * Y[(1 * PP + sn) * SP + lb];
    X[(3 * PP + s) * SP + lb] = dz - az * dhl - czz * Y[(2 * PP + sn) * SP + lb];
  }
  __syncthreads();  // separator rows
  // transposed: thread (line lt, separator st) in PP consecutive lanes
  {
    const int lt = tid / PP, st = tid % PP;
    const int lane = tid & 63, grp = lane - st;
    T ra = 0, rb = 1, rg = 0, rd = 0;
    if (lt < TL && st < P) {
      ra = X[(0 * PP + st) * SP + lt];
      rb = X[(1 * PP + st) * SP + lt];
      rg = X[(2 * PP + st) * SP + lt];
      rd = X[(3 * PP + st) * SP + lt];
    }
    for (int step = 1; step < PP; step <<= 1) {
      int im = st - step, ip = st + step;
      bool hm = true, hp = true;
      if (K.cyc) {
        im &= PP - 1;
        ip &= PP - 1;
      } else {
        hm = im >= 0;
        hp = ip < PP;
      }
      const int sm_ = grp + (hm ? im : st), sp_ = grp + (hp ? ip : st);
      T am = lane_read(ra, sm_), bm = lane_read(rb, sm_), gm = lane_read(rg, sm_),
        dm = lane_read(rd, sm_);
      T ap = lane_read(ra, sp_), bp = lane_read(rb, sp_), gp = lane_read(rg, sp_),
        dp = lane_read(rd, sp_);
      if (!hm) {
        am = 0;
        bm = 1;
        gm = 0;
        dm = 0;
      }
      if (!hp) {
        ap = 0;
        bp = 1;
        gp = 0;
        dp = 0;
      }
      const T k1 = ra / bm, k2 = rg / bp;
      const T na = -am * k1, ng = -gp * k2;
      rb = rb - gm * k1 - ap * k2;
      rd = rd - dm * k1 - dp * k2;
      ra = na;
      rg = ng;
    }
    if (lt < TL && st < P) Y[st * SP + lt] = K.cyc ? rd / (ra + rb + rg) : rd / rb;
  }
  if (UPRE && active) {
    // the velocity the solution is added to: loaded here, where the
    // registers of the separator solve are free, in flight over the barrier
#pragma unroll
    for (int e = 0; e < NPRE; ++e) uu[e] = buf_ld<double>(ures, vline * 8u, (uint32_t)e * rstride * 8u);
  }
  __syncthreads();  // separator values
  if (active) {
    const T zr = Y[s * SP + lb];
    const T zl = (s > 0) ? Y[(s - 1) * SP + lb] : (K.cyc ? Y[(P - 1) * SP + lb] : T(0));
    if (!rare) {
#pragma unroll
      for (int e = 0; e < m; ++e) dd[e] = dd[e] - CTAB(2, e) * zl - CTAB(3, e) * zr;
      dd[m] = zr;
#pragma unroll
      for (int e = 0; e < SL; ++e) {
        if (MODE == 2)
          buf_st(u_at(e) + (double)dd[e], ures, vline * 8u, (uint32_t)e * rstride * 8u);
        else
          buf_st(dd[e], dres, vlb, roff(e));
      }
    } else {
      // the rare path again: rows and coefficients from memory, RC at a time
#pragma unroll
      for (int e0 = 0; e0 < SL; e0 += RC) {
        __builtin_amdgcn_sched_barrier(0);
        T ca[RC], cc[RC], cd[RC];
#pragma unroll
        for (int q = 0; q < RC; ++q)
          if (e0 + q < m) {
            ca[q] = buf_ld<T>(sares, vlb, roff(e0 + q));
            cc[q] = buf_ld<T>(scres, vlb, roff(e0 + q));
            cd[q] = buf_ld<T>(dres, vlb, roff(e0 + q));
          }
#pragma unroll
        for (int q = 0; q < RC; ++q) {
          const int e = e0 + q;
          if (e < SL) {
            const T x = (e < m) ? cd[q] - ca[q] * zl - cc[q] * zr : zr;
            if (MODE == 2)
              buf_st(u_at(e) + (double)x, ures, vline * 8u, (uint32_t)e * rstride * 8u);
            else
              buf_st(x, dres, vlb, roff(e));
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#undef CTAB
  }
}

template <typename T>
static void launch_line(Prof* pf, hipStream_t s, LineK<T> K, const char* name) {
  dim3 grid;
  int threads;
  if (K.mode == 0) {
    K.tl = 256 / K.P;
    threads = K.tl * K.P;
    const int64_t rows = (int64_t)K.nj * K.nz;
    grid = dim3((unsigned)((rows + K.tl - 1) / K.tl));
  } else {
    // 16 consecutive lines per block whenever the segments allow (a
    // wavefront's loads then cover 128-byte row pieces), up to 1024 threads
    K.tl = 1024 / K.P;
    if (K.tl > 16) K.tl = 16;
    if (K.tl < 1) K.tl = 1;
    threads = K.tl * K.P;
    grid = dim3((K.nx + K.tl - 1) / K.tl, K.mode == 1 ? K.nj : K.nz);
  }
  size_t work = 8 * (size_t)K.P * K.tl;  // separator arrays
  if (K.mode == 0) {                      // x sweep: also the staged rows
    const size_t rows = (size_t)K.tl * (K.n + (K.n >> 4) + 1);
    if (rows > work) work = rows;
  }
  K.tab1 = (K.mode != 2 && K.r == 0) ? 1 : 0;
  const size_t shm = sizeof(T) * (LINE_NTAB * (size_t)(K.tab1 ? 1 : K.P) * LMAX + work);
  // fixed-length segments only for the x sweep: unrolled strided z/y
  // segments need ~190 VGPRs (2 waves per SIMD), slower than the ragged form
  const bool fixed = (K.mode == 0 && K.r == 0 && K.L == LMAX);
#define IBM_LINE(M)                                                                   \
  do {                                                                                \
    if (fixed)                                                                        \
      IBM_LAUNCH_G(pf, name, s, (&k_line<T, M, true, true>), dim3(grid), dim3(threads), shm, K, k_line<T, M, true><<<grid, threads, shm, s>>>(K));   \
    else                                                                              \
      IBM_LAUNCH_G(pf, name, s, (&k_line<T, M, false, true>), dim3(grid), dim3(threads), shm, K, k_line<T, M, false><<<grid, threads, shm, s>>>(K));  \
  } while (0)
  if (K.mode == 0 && fixed && (K.P & (K.P - 1)) == 0 && K.P >= 4 && K.P <= 64) {
    // one wavefront per group of 64/P rows, four wavefronts per block, as
    // many blocks as are resident at once (each wavefront loops over groups)
    const int64_t rows = (int64_t)K.nj * K.nz;
    const int64_t waves = (rows + 64 / K.P - 1) / (64 / K.P);
    const size_t xshm = sizeof(T) * (LINE_NTAB * LMAX + 4 * 64 * (size_t)(LMAX + 16 / sizeof(T)));
    static int resident = 0;  // per element type: the shared memory size is fixed
    if (resident == 0) {
      int dev = 0, cus = 0, per = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_line_xw<T>, 256, xshm) != hipSuccess ||
          cus < 1 || per < 1)
        cus = 256, per = 1;
      resident = cus * per;
    }
    int64_t blocks = (waves + 3) / 4;
    if (blocks > resident) blocks = resident;
    IBM_LAUNCH_G(pf, name, s, (&k_line_xw<T, true>), dim3((unsigned)blocks), dim3(256), xshm, K, k_line_xw<T><<<(unsigned)blocks, 256, xshm, s>>>(K));
  } else if (K.mode == 0) {
    IBM_LINE(0);
  } else if (K.r == 0 &&
             (K.L == LMAX || (K.mode == 2 && (K.L == 12 || K.L == 24)) ||
              (K.mode == 1 && K.L == 32)) &&
             K.nx % (K.L > LMAX ? 32 : 16) == 0 && K.P <= 64 &&
             (!K.cyc || (K.P & (K.P - 1)) == 0) &&
             (K.mode == 1 ? (int64_t)K.nx : K.plane) * 64 * 8 < ((int64_t)1 << 31)) {
    // column sweep: 16 lines per block (32 in FP32 where the block stays
    // within 1024 threads, and with the long segments of the large planes),
    // the separators solved per wavefront; a wavefront's rows (at most 64)
    // span less than 2 GiB of any array, the range of its buffer descriptors
    int pp = 1;
    while (pp < K.P) pp <<= 1;
    K.PP = pp;
    const int tl = (K.L > LMAX || (sizeof(T) == sizeof(float) && pp <= 32 && K.nx % 32 == 0))
                       ? 32 : 16;
    const int ct = tl * pp;
    const size_t cshm = sizeof(T) * (LINE_NTAB * (size_t)(K.tab1 ? 1 : K.P) * K.L +
                                     7 * (size_t)pp * (tl + 1)) +
                        sizeof(uint32_t) * (size_t)K.P * K.L +
                        ((K.mode == 2 && K.L > LMAX) ? sizeof(T) * 3 * (size_t)K.P * K.L : 0);
    // whole rows or planes per XCD in a 1-D grid (see the kernels); the
    // register kernel keeps its z-major 2-D grid on planes below 512 x 512,
    // where the 1-D order measured slower
    const int nout = (K.mode == 2) ? K.nz : K.nj;
    const dim3 lgrid((unsigned)(NUM_XCD * ((nout + NUM_XCD - 1) / NUM_XCD) * (K.nx / tl)));
    K.xrow = (int64_t)K.nx * K.nz >= 512 * 512;
    const dim3 rgrid = K.xrow ? lgrid : dim3(K.nz, K.nx / tl);
#define IBM_COL(M, SL_, KERN, GRID)                                                            \
  do {                                                                                        \
    if constexpr (sizeof(T) == sizeof(float)) {                                               \
      if (tl == 32) {                                                                         \
        IBM_LAUNCH_G(pf, name, s, (&KERN<T, M, SL_, 32, true>), dim3(GRID), dim3(ct), cshm, K, \
                     KERN<T, M, SL_, 32><<<GRID, ct, cshm, s>>>(K));                          \
        break;                                                                                \
      }                                                                                       \
    }                                                                                         \
    IBM_LAUNCH_G(pf, name, s, (&KERN<T, M, SL_, 16, true>), dim3(GRID), dim3(ct), cshm, K,    \
                 KERN<T, M, SL_, 16><<<GRID, ct, cshm, s>>>(K));                              \
  } while (0)
    if constexpr (sizeof(T) == sizeof(float)) {  // the long segments (FP32 plans only)
      if (K.L == 32) {
        IBM_LAUNCH_G(pf, name, s, (&k_line_col<T, 1, 32, 32, true>), lgrid, dim3(ct), cshm, K,
                     k_line_col<T, 1, 32, 32><<<lgrid, ct, cshm, s>>>(K));
        return;
      }
      if (K.L == 24) {
        IBM_LAUNCH_G(pf, name, s, (&k_line_col<T, 2, 24, 32, true>), lgrid, dim3(ct), cshm, K,
                     k_line_col<T, 2, 24, 32><<<lgrid, ct, cshm, s>>>(K));
        return;
      }
    }
    // wall-normal lines of 12 or 16 rows: the register form
    if (K.mode == 1)
      IBM_COL(1, LMAX, k_line_col, lgrid);
    else if (K.L == 12)
      IBM_COL(2, 12, k_line_col_reg, rgrid);
    else
      IBM_COL(2, LMAX, k_line_col_reg, rgrid);
#undef IBM_COL
  }
  else if (K.mode == 1)
    IBM_LAUNCH_G(pf, name, s, (&k_line<T, 1, false, true>), dim3(grid), dim3(threads), shm, K, k_line<T, 1, false><<<grid, threads, shm, s>>>(K));
  else
    IBM_LAUNCH_G(pf, name, s, (&k_line<T, 2, false, true>), dim3(grid), dim3(threads), shm, K, k_line<T, 2, false><<<grid, threads, shm, s>>>(K));
#undef IBM_LINE
}

template <typename T>
static LineK<T> base_k(const GridView& g, void* d, const uint32_t* mask, void* sa, void* sc) {
  LineK<T> K{};
  K.d = static_cast<T*>(d);
  K.mask = mask;
  K.sa = static_cast<T*>(sa);
  K.sc = static_cast<T*>(sc);
  K.nx = g.nx;
  K.nz = g.nz;
  K.plane = (int64_t)g.nz * g.nx;
  return K;
}

template <typename T>
static void adi_periodic(Prof* pf, hipStream_t s, const GridView& g, int comp, int mode, void* d,
                         const uint32_t* mask, const CyclicTab& t, void* sa, void* sc) {
  LineK<T> K = base_k<T>(g, d, mask, sa, sc);
  K.tab = static_cast<const T*>(sizeof(T) == sizeof(float) ? (const void*)t.seg32 : (const void*)t.seg);
  K.mode = mode;
  K.n = (mode == 0) ? g.nx : g.nz;
  K.cyc = 1;
  line_plan(K.n, true, mode == 0 ? LINE_LMAX : z_seg_len(K.n, g.nx, sizeof(T) == sizeof(float)),
            &K.P, &K.L, &K.r);
  K.a = (T)t.a;
  K.b = (T)t.b;
  K.c = (T)t.c;
  K.j0 = (comp == 1) ? 1 : 0;
  K.nj = (comp == 1) ? g.ny - 1 : g.ny;
  launch_line(pf, s, K, mode == 0 ? "adi_x" : "adi_z");
}

void launch_adi_x(Prof* pf, hipStream_t s, const GridView& g, int comp, void* d,
                  const uint32_t* mask, const CyclicTab& t, void* sa, void* sc, int fp32) {
  if (fp32)
    adi_periodic<float>(pf, s, g, comp, 0, d, mask, t, sa, sc);
  else
    adi_periodic<double>(pf, s, g, comp, 0, d, mask, t, sa, sc);
}

void launch_adi_z(Prof* pf, hipStream_t s, const GridView& g, int comp, void* d,
                  const uint32_t* mask, const CyclicTab& t, void* sa, void* sc, int fp32) {
  if (fp32)
    adi_periodic<float>(pf, s, g, comp, 1, d, mask, t, sa, sc);
  else
    adi_periodic<double>(pf, s, g, comp, 1, d, mask, t, sa, sc);
}

template <typename T>
static void adi_wall(Prof* pf, hipStream_t s, const GridView& g, void* d, double* u,
                     const uint32_t* mask, const YTab& t, void* sa, void* sc) {
  LineK<T> K = base_k<T>(g, d, mask, sa, sc);
  const bool f = sizeof(T) == sizeof(float);
  K.tab = static_cast<const T*>(f ? (const void*)t.seg32 : (const void*)t.seg);
  K.mode = 2;
  K.u = u;
  K.n = t.n;
  K.cyc = 0;
  line_plan(K.n, false, wall_seg_len(K.n, g.nx, sizeof(T) == sizeof(float)), &K.P, &K.L, &K.r);
  K.A = static_cast<const T*>(f ? (const void*)t.a32 : (const void*)t.a);
  K.B = static_cast<const T*>(f ? (const void*)t.b32 : (const void*)t.b);
  K.C = static_cast<const T*>(f ? (const void*)t.c32 : (const void*)t.c);
  K.j0 = t.j0;
  K.nj = t.n;
  launch_line(pf, s, K, "adi_y");
}

void launch_adi_y(Prof* pf, hipStream_t s, const GridView& g, int comp, void* d, double* u,
                  const uint32_t* mask, const YTab& t, void* sa, void* sc, int fp32) {
  (void)comp;
  if (fp32)
    adi_wall<float>(pf, s, g, d, u, mask, t, sa, sc);
  else
    adi_wall<double>(pf, s, g, d, u, mask, t, sa, sc);
}

}  // namespace ibm
