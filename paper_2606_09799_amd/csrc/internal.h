// Internal declarations shared by the HIP translation units of libibm.
// Not part of the public ABI (include/ibm.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace ibm {

typedef unsigned long long u64;

// Grid metrics as seen by the kernels (all device pointers).  The y lattice of
// a component including its two wall points ("ext"): u and w use extuw
// (ny+2 heights: yf[0], yc[0..ny-1], yf[ny]; node j <-> ext index j+1); v uses
// yf (ny+1 heights; node j <-> ext index j).
struct GridView {
  int nx, ny, nz, nxh;  // nxh = nx/2 + 1 (half spectrum)
  double dx, dz, lx, lz;
  double dmax;          // largest same-lattice neighbour distance
  const double* yf;     // ny+1
  const double* yc;     // ny
  const double* dy;     // ny
  const double* dyc;    // ny+1
  const double* extuw;  // ny+2
  // reciprocals and interpolation weights (host-computed; no division in the
  // stencil kernels)
  double idx, idz;      // 1/dx, 1/dz
  const double* idy;    // ny: 1/dy[j]
  const double* idyc;   // ny+1: 1/dyc[j]
  const double* fw0;    // ny+1: face f value = a[f-1] fw0[f] + a[f] fw1[f]
  const double* fw1;    //       (f = 1..ny-1; 0 at the walls)
};

struct BodyDev {
  const double* xyz;
  const double* vel;
  const int32_t* tri;
  int32_t nt;
  int32_t toff;  // global id of the body's first triangle
};
inline bool operator==(const BodyDev& a, const BodyDev& b) {
  return a.xyz == b.xyz && a.vel == b.vel && a.tri == b.tri && a.nt == b.nt && a.toff == b.toff;
}

// Coefficient tables of the three line-solve directions for one beta
// (device arrays).  Cyclic x/z: the Thomas factorisation of the matrix with
// its corners removed (Sherman-Morrison form), the weights W that give
// y_0 = sum_i W_i d'_i during the forward sweep, and z = T^{-1} u.
struct CyclicTab {
  const double* cp;
  const double* inv;
  const double* W;
  const double* Z;
  double a, b, c;        // constant sub/main/super diagonal
  double ratio;          // beta_corner / gamma
  double fden_inv;       // 1 / (1 + z_0 + ratio z_{n-1})
  const double* seg;     // partitioned-solve tables [LINE_NTAB][P][LINE_TLD]
  const float* seg32;    // the same tables in FP32 (mixed form)
};

struct YTab {
  // rows r = 0..n-1 of the wall-normal system of one lattice (n = ny; u/w:
  // row r <-> node j = r; v: row r <-> face j = r+1, the last row being the
  // top wall face as an identity row)
  const double* a;   // sub-diagonal
  const double* b;   // diagonal
  const double* c;   // super-diagonal
  const double* cp;  // Thomas c' of the mask-free system
  const double* inv; // 1/pivot of the mask-free system
  const double* seg; // partitioned-solve tables [LINE_NTAB][P][LINE_TLD]
  // FP32 copies of a, b, c and seg (mixed form)
  const float *a32, *b32, *c32, *seg32;
  int n, j0;
};

// Segmentation of a line of n rows for the partitioned solves: P balanced
// segments of at most lmax rows (the first r segments hold L+1 rows, the
// others L); cyclic lines use at least 3 segments.  Shared by the kernels
// and the host code that builds their tables.  The mask-free elimination
// tables hold LINE_TLD entries per segment whatever its length.
constexpr int LINE_LMAX = 16;
constexpr int LINE_TLD = 32;
constexpr int LINE_NTAB = 5;  // tables per segment row (see the partitioned solve)
inline void line_plan(int n, bool cyc, int lmax, int* P, int* L, int* r) {
  int p = (n + lmax - 1) / lmax;
  if (cyc && p < 3) p = 3;
  *P = p;
  *L = n / p;
  *r = n % p;
}
inline void line_plan(int n, bool cyc, int* P, int* L, int* r) {
  line_plan(n, cyc, LINE_LMAX, P, L, r);
}
inline bool pow2_in(int p, int lo, int hi) { return p >= lo && p <= hi && (p & (p - 1)) == 0; }
// Segment length of the wall-normal lines (nx x-points per line row): 12
// rows where that cuts a line of n rows into a power of two of segments (4
// to 64: the separator reduction then has no idle lanes, and the
// per-thread arrays are shorter); 24 rows where 12-row segments would number
// 64 and 24-row ones a power of two (32 lines per block instead of 16, so
// that each row access of a block covers twice the bytes of one plane: on
// large planes every row of a line lies in another page; FP32 line data
// only, the FP64 solve would not fit its registers); else LINE_LMAX.  The
// tables and the launch both take their plan from here.
inline int wall_seg_len(int n, int nx, bool fp32) {
  if (fp32 && n % 24 == 0 && n / 12 == 64 && nx % 32 == 0) return 24;
  if (n % 12 == 0 && pow2_in(n / 12, 4, 64)) return 12;
  return LINE_LMAX;
}
// Segment length of the periodic z lines: 32 rows where 16-row segments
// would number more than 32 and 32-row ones a power of two (32 lines per
// block instead of 16: 128-byte row pieces; FP32 line data only, as above),
// else LINE_LMAX.
inline int z_seg_len(int n, int nx, bool fp32) {
  if (fp32 && n % 32 == 0 && n / 16 > 32 && pow2_in(n / 32, 4, 32) && nx % 32 == 0) return 32;
  return LINE_LMAX;
}

// Row stride (complex values) of the half spectrum [y][z][mode]: nx/2+1
// modes padded to a multiple of 128 bytes, so that the z transforms' tiles of
// consecutive modes start on cache-line boundaries
inline int spec_ld(int nxh, bool fp32) {
  const int a = fp32 ? 16 : 8;
  return (nxh + a - 1) / a * a;
}

struct FFTPlan {
  int n;
  int nst;
  int radix[16];
  const double2* tw;  // exp(-2 pi i k/n), k = 0..n-1
  const float2* tw32; // the same, rounded to FP32
};

// Stages of the mixed-radix transforms of length n (radices 4, 2, 3, 5, 7,
// a 2 only where no 4 remains); false if n has another prime factor.  The
// twiddle pointers are left to the caller.
inline bool plan_fft(int n, FFTPlan* P) {
  P->n = n;
  P->nst = 0;
  int m = n;
  const int radices[5] = {4, 2, 3, 5, 7};
  for (int r : radices) {
    while (m % r == 0) {
      if (r == 2 && m % 4 == 0) break;
      if (P->nst >= 16) return false;
      P->radix[P->nst++] = r;
      m /= r;
    }
  }
  return m == 1;
}

// blocks of the XCD band order (lanes.h: xcd_band_tile), bands of BW k-tiles
inline int64_t xcd_band_blocks(int nbx, int nbz, int ny, int BW) {
  const int64_t bands = (nbz + BW - 1) / BW;
  return 8 * ((bands + 7) / 8) * (int64_t)nbx * BW * ny;
}

// profiling hook (ctx.cpp): an event pair around each kernel launch when
// profiling is enabled and the kernel name matches the filter
struct Prof;
void prof_begin(Prof* p, const char* name, hipStream_t s);
void prof_end(Prof* p, hipStream_t s);

// Launch recording (the grouped batched form).  While a recorder is set on
// this host thread, a launch that has a grouped form is appended to it
// instead of being issued: the grouped instantiation of its kernel, its
// argument record, grid, block and dynamic LDS size.  A launch without a
// grouped form marks the recording unusable (the batch then keeps its
// stream plans).
struct LaunchRec {
  const char* name;
  const void* gfunc;
  std::vector<unsigned char> arg;
  dim3 grid, block;
  size_t shm;
};
struct Recorder {
  std::vector<LaunchRec> recs;
  bool bad = false;
};
// The argument of a kernel's grouped instantiation: the members' argument
// records (ksize bytes each), their block offsets (n + 1 prefix sums), their
// grids (3 per member) and the member of every block of the launch, all in
// device memory.
struct GrpTab {
  const unsigned char* k;
  const uint32_t* boff;
  const uint32_t* gdim;
  const uint16_t* bm;
  int n;
  int ksize;
};
Recorder*& cur_recorder();
void record_launch(const char* name, const void* gfunc, dim3 grid, dim3 block, size_t shm,
                   const void* arg, size_t bytes);

#define IBM_LAUNCH(pf, name, s, ...)          \
  do {                                        \
    if (::ibm::cur_recorder()) {              \
      ::ibm::cur_recorder()->bad = true;      \
    } else {                                  \
      ::ibm::prof_begin(pf, name, s);         \
      __VA_ARGS__;                            \
      ::ibm::prof_end(pf, s);                 \
    }                                         \
  } while (0)
// A launch with a grouped form: GF is the address of the kernel's grouped
// instantiation (in parentheses), K its single argument; the launch
// expression follows.
#define IBM_LAUNCH_G(pf, name, s, GF, GRID, BLOCK, SHM, K, ...)                       \
  do {                                                                               \
    if (::ibm::cur_recorder()) {                                                     \
      ::ibm::record_launch(name, (const void*)GF, GRID, BLOCK, SHM, &(K), sizeof(K)); \
    } else {                                                                         \
      ::ibm::prof_begin(pf, name, s);                                                \
      __VA_ARGS__;                                                                   \
      ::ibm::prof_end(pf, s);                                                        \
    }                                                                                \
  } while (0)

// sticky flags (same bits as IBM_FLAG_*)
constexpr uint32_t FLAG_CAPACITY = 1u, FLAG_NONFINITE = 2u, FLAG_GEOM = 4u, FLAG_REFINE = 8u,
                   FLAG_CFL = 16u, FLAG_COMPAT = 32u;

// ------------------------------------------------------------ launchers
// body.hip
void launch_body_rigid(Prof* pf, hipStream_t s, const double* x0, int nv, const double* coef,
                       double* xyz, double* vel);
void launch_body_deform(Prof* pf, hipStream_t s, const double* data, int nv, const double* coef,
                        double* xyz, double* vel);
// the same transforms with the coefficients in device memory (rigid: 18
// values, deform: 6, the layouts of the host calls)
void launch_body_dev(Prof* pf, hipStream_t s, int deform, const double* ref, int nv,
                     const double* coef_dev, double* xyz, double* vel);

// tag.hip
struct TagBuffers {
  uint32_t* mask[3];
  u64* best_d[3];
  int32_t* best_t[3];
  int64_t* idx[3];
  int32_t* tri[3];
  int64_t* cb;
  uint32_t* cb_mask;
  int64_t* count;        // [4]
  int64_t* block_sums;   // scan scratch: 3 regions of bsum_stride values
  int64_t bsum_stride;
  int64_t cap;
  int64_t nwords[3];     // mask words per component
  int64_t nwords_cb;
};
// dt > 0: also flags (FLAG_CFL) a vertex whose velocity carries it more than
// half the local spacing along an axis in dt
void launch_tag(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nbody,
                int ntri, TagBuffers& tb, uint32_t* flags, double dt);

// force.hip
// pressure reconstructed on the boundary cells of tb (p: FP32 when fp32),
// out[f] for the f-th cell of the C_B list (at most out_cap values)
void launch_pressure_cb(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies,
                        int nbody, const TagBuffers& tb, const void* p, int fp32, double* out,
                        int64_t out_cap, uint32_t* flags);
// no-slip error of the fields at the forcing nodes of tb: per-node errors in
// vals (3 * cap), per-component means in out[3] (device)
void launch_noslip(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nbody,
                   const TagBuffers& tb, const double* const* fields, double* vals, double* out,
                   uint32_t* flags);
void launch_force(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nbody,
                  const TagBuffers& tb, double* const* fields, double* vals,
                  uint32_t* flags);

// rhs.hip
// p, hprev, hout and R are FP64, or FP32 when fp32 is set (mixed form)
struct RhsArgs {
  const double *u, *v, *w;
  const void* p;
  const void* hprev[3];
  void* hout[3];
  void* R[3];
  const uint32_t* mask[3];
  double gamma, rho, alpha, dt, re, fx;
  int fp32;
  int planes;  // wall-normal planes per block of the march (1..64; 0: the default)
};
void launch_rhs(Prof* pf, hipStream_t s, const GridView& g, const RhsArgs& a);
// volume force of component comp: R += adt (f0 + kappa u) on its unknown
// nodes that are not forcing nodes (f0, kappa: NULL = 0)
void launch_vforce(Prof* pf, hipStream_t s, const GridView& g, int comp, void* R, int fp32,
                   const uint32_t* mask, const double* u, const double* f0, const double* kappa,
                   double adt);

// adi.hip
// d, sa, sc: FP64, or FP32 when fp32 is set.  sa, sc: scratch of the size of
// the field (used only by segments that hold forcing nodes)
void launch_adi_x(Prof* pf, hipStream_t s, const GridView& g, int comp, void* d,
                  const uint32_t* mask, const CyclicTab& t, void* sa, void* sc, int fp32);
void launch_adi_z(Prof* pf, hipStream_t s, const GridView& g, int comp, void* d,
                  const uint32_t* mask, const CyclicTab& t, void* sa, void* sc, int fp32);
void launch_adi_y(Prof* pf, hipStream_t s, const GridView& g, int comp, void* d, double* u,
                  const uint32_t* mask, const YTab& t, void* sa, void* sc, int fp32);

// mass.hip
void launch_mass(Prof* pf, hipStream_t s, const GridView& g, const double* u, const double* v,
                 const double* w, const int64_t* cb, const int64_t* count, int64_t cap,
                 double vtot, int use_q, double* partial, double* qf, uint32_t* flags);
void launch_mass_rhs(Prof* pf, hipStream_t s, const GridView& g, const double* u, const double* v,
                     const double* w, const uint32_t* cb_mask, const double* qf,
                     double inv_adt, double* rhs);

// max over C_F of |D u - qf[0]| into *out (partial: 256 doubles)
void launch_divergence(Prof* pf, hipStream_t s, const GridView& g, const double* u,
                       const double* v, const double* w, const uint32_t* cb_mask,
                       const double* qf, double* partial, double* out);
// compatibility of a Neumann right-hand side: FLAG_COMPAT when
// |sum rhs dV| > 1e-12 sum |rhs| dV (fixed-order sums; partial: 512 doubles)
void launch_compat(Prof* pf, hipStream_t s, const GridView& g, const double* rhs,
                   double* partial, uint32_t* flags);

// mass- and energy-conserving q_F (App. B): qcoef[0..1] = (c0, c1) with
// q_F = c0 + c1 (p - e); partial: 5 * 512 doubles; p: FP64, or FP32 when fp32
void launch_mass_energy(Prof* pf, hipStream_t s, const GridView& g, const double* u,
                        const double* v, const double* w, const void* p, int fp32,
                        const uint32_t* cb_mask, double* partial, double* qcoef,
                        uint32_t* flags);
void launch_mass_rhs_energy(Prof* pf, hipStream_t s, const GridView& g, const double* u,
                            const double* v, const double* w, const void* p, int fp32,
                            const uint32_t* cb_mask, const double* qcoef, double inv_adt,
                            double* rhs);

// poisson.hip
struct PoissonArgs {
  const FFTPlan* px;   // length nx (host copy of the plan, tables on device)
  const FFTPlan* pz;   // length nz
  const double* lamx;  // nxh
  const double* lamz;  // nz
  const double* ylo;   // ny: coefficient of phi[j-1]
  const double* yhi;   // ny: coefficient of phi[j+1]
  void* spec;          // ny*nz*spec_ld(nxh) complex: double2, or float2 when fp32
  void* spec64;        // refined mixed form: the FP64 spectrum written by the wall-normal
                       // solve and read by FP64 inverse passes (NULL: inverse passes on spec)
  double sum_dy;
  int fp32;            // FP32 spectrum and transforms
  int p_fp32;          // the pressure (read by the energy-conserving q) is FP32
  // FP64-residual refinement (mixed form)
  int refine;          // on/off
  int nref;            // refinements at most
  double tol;          // bound on max|rhs - L_c phi| * alpha dt
  double* rhs_keep;    // N: FP64 right-hand side kept for the residuals
  u64* rmax;           // nref + 2 slots
  double* stats;       // [solves, corrections, largest final residual]
  double* zm;          // ny: the (0,0) mode column in FP64 (FP32 spectrum)
  double* psum;        // per-block partial sums (x-pass blocks)
  double* msum;        // nref + 2: sum of phi dV at each refinement
  double vtot;         // volume of the box
  uint32_t* flags;
};
// rhs from an array (rhs != NULL) or formed on the fly from the velocity
// (rhs == NULL): (D u - q)/alpha_dt on C_F, 0 on C_B, with q = qf[0], or
// q = qf[0] + qf[1] (p - e) when p != NULL (the energy-conserving shape; p
// FP32 when a.p_fp32)
void launch_poisson(Prof* pf, hipStream_t s, const GridView& g, const PoissonArgs& a,
                    const double* rhs, const double* u, const double* v, const double* w,
                    const uint32_t* cb_mask, const double* qf, const void* p, double inv_adt,
                    double* phi);

// project.hip
// p: FP64, or FP32 when fp32 is set
void launch_project(Prof* pf, hipStream_t s, const GridView& g, const double* phi, double adt,
                    double re, double* u, double* v, double* w, void* p, int fp32);

// hydrodynamic loads (loads.hip): per-marker tractions (3 ntri) and per-body
// force and torque about pole (6 nb) of the bodies of the last tagging
void launch_loads(Prof* pf, hipStream_t s, const GridView& g, const BodyDev* bodies, int nb,
                  int ntri, const double* u, const double* v, const double* w, const void* p,
                  int p32, const uint32_t* cb_mask, const int32_t* sides, const double* pole,
                  double re, double* traction, double* loads);

// rigid-body dynamics (rigid.hip): one AB2 step per body, coefficients out
void launch_rigid_advance(Prof* pf, hipStream_t s, int nb, double* state, const double* props,
                          const double* loads, double dt, double* coef);

// utilities (util.hip)
void launch_fill_u32(Prof* pf, hipStream_t s, uint32_t* p, int64_t n, uint32_t val);
void launch_fill_u8(Prof* pf, hipStream_t s, uint8_t* p, int64_t n, uint8_t val);
void launch_fill_u64(Prof* pf, hipStream_t s, u64* p, int64_t n, u64 val);
void launch_fill_i32(Prof* pf, hipStream_t s, int32_t* p, int64_t n, int32_t val);
void launch_fill_f64(Prof* pf, hipStream_t s, double* p, int64_t n, double val);


}  // namespace ibm
