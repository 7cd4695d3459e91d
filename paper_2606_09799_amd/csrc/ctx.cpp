// Host side of libibm: the context (grid metrics, workspace, line-solve and
// FFT tables), the orchestration of one time step on one HIP stream, the
// sticky error word, per-kernel event timing, and the exported C-ABI of
// include/ibm.h.  Every call only enqueues work; nothing synchronises except
// ibm_check, ibm_tags_count_host and ibm_profile_read.
#include "ibm.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace ibm;

static thread_local std::string g_last_error;

#define HIPCHK(expr)                                                       \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(e_);   \
      return IBM_EHIP;                                                     \
    }                                                                      \
  } while (0)

// ------------------------------------------------------------ recording
namespace ibm {
Recorder*& cur_recorder() {
  static thread_local Recorder* r = nullptr;
  return r;
}

void record_launch(const char* name, const void* gfunc, dim3 grid, dim3 block, size_t shm,
                   const void* arg, size_t bytes) {
  Recorder* r = cur_recorder();
  LaunchRec e;
  e.name = name;
  e.gfunc = gfunc;
  e.arg.assign(static_cast<const unsigned char*>(arg), static_cast<const unsigned char*>(arg) + bytes);
  e.grid = grid;
  e.block = block;
  e.shm = shm;
  r->recs.push_back(std::move(e));
}

// ------------------------------------------------------------ profiling
struct Prof {
  bool enabled = false;
  std::string filter;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  bool open = false;

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};

void prof_begin(Prof* p, const char* name, hipStream_t s) {
  if (!p || !p->enabled) return;
  if (!p->filter.empty() && std::strstr(name, p->filter.c_str()) == nullptr) return;
  Prof::Rec r{name, p->take(), p->take()};
  (void)hipEventRecord(r.a, s);
  p->recs.push_back(r);
  p->open = true;
}

void prof_end(Prof* p, hipStream_t s) {
  if (!p || !p->open) return;
  (void)hipEventRecord(p->recs.back().b, s);
  p->open = false;
}
}  // namespace ibm

// ------------------------------------------------------------ context
struct ibm_ctx {
  int dev = 0;
  int rhs_planes = 0;  // planes per block of the RHS march (0: the default)
  hipStream_t stream = nullptr;
  int nx = 0, ny = 0, nz = 0;
  double lx = 0, lz = 0;
  ibm_opts opts{};
  int64_t ncell = 0, nvface = 0;
  std::vector<double> yf, yc, dy, dyc, extuw;
  GridView g{};
  std::vector<void*> allocs;

  TagBuffers tb{};
  double* force_vals = nullptr;
  std::vector<BodyDev> bodies;  // bodies of the last ibm_tag
  std::vector<BodyDev> last_bodies;
  int ntri = 0;
  static constexpr int NSLOT = 8;
  static constexpr int MAXB = 128;  // bodies per context
  BodyDev* dslots = nullptr;  // NSLOT x MAXB descriptors (device)
  BodyDev* hslots = nullptr;  // NSLOT x MAXB descriptors (pinned host)
  hipEvent_t slot_ev[NSLOT] = {};
  bool slot_used[NSLOT] = {};
  int cur_slot = -1;
  const BodyDev* d_bodies = nullptr;

  // precision of the predictor and spectral work: FP64, or FP32 in the mixed
  // form (element size es); the velocity and phi are FP64 in both
  int fp32 = 0;
  int pfp32 = 0;  // mixed form: FP32 Poisson transforms with FP64-residual refinement
  size_t es = sizeof(double);
  void* R[3] = {};
  void* H[3] = {};
  void* sa = nullptr;  // line-solve scratch (segments with forcing nodes)
  void* sc = nullptr;
  double* phi = nullptr;
  void* spec = nullptr;
  // refined mixed form: the FP64 spectrum of the inverse passes
  void* spec64 = nullptr;
  // mixed form: FP64-residual refinement of the Poisson solve
  double* rhs_keep = nullptr;
  // volume force per component (caller's arrays): f0 + kappa u_c
  const double* vf0[3] = {nullptr, nullptr, nullptr};
  const double* vkap[3] = {nullptr, nullptr, nullptr};
  u64* rmax = nullptr;
  double* rstats = nullptr;
  double* zm = nullptr;
  double* psum = nullptr;
  double* msum = nullptr;
  int nref = 0;
  double rtol = 0.0;
  double* partial = nullptr;
  double* qf = nullptr;
  double* diag = nullptr;  // per-component no-slip errors (3)
  uint32_t* flags = nullptr;

  // line-solve tables for one beta; a new beta is staged through a ring of
  // pinned host slots and copied in stream order (no synchronisation)
  double tab_beta = -1.0;
  double* tabmem = nullptr;
  float* tabmem32 = nullptr;
  int64_t tabcap = 0;
  static constexpr int NTSTAGE = 4;
  double* tab_host[NTSTAGE] = {};
  float* tab_host32[NTSTAGE] = {};
  hipEvent_t tab_ev[NTSTAGE] = {};
  bool tab_used[NTSTAGE] = {};
  int tab_stage = 0;
  CyclicTab ctx_x{}, ctx_z{};
  YTab yt[2]{};  // 0: u and w, 1: v

  // Poisson
  FFTPlan px{}, pz{};
  double* lamx = nullptr;
  double* lamz = nullptr;
  double* ylo = nullptr;
  double* yhi = nullptr;
  double sum_dy = 0, vtot = 0;

  Prof prof;
};

template <typename T>
static int dalloc(ibm_ctx* c, T** p, int64_t n) {
  void* q = nullptr;
  size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    g_last_error = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    return IBM_ENOMEM;
  }
  c->allocs.push_back(q);
  *p = (T*)q;
  return IBM_OK;
}

static int dalloc_bytes(ibm_ctx* c, void** p, int64_t n, size_t es) {
  char* q = nullptr;
  int rc = dalloc(c, &q, n * (int64_t)es);
  *p = q;
  return rc;
}

template <typename T>
static int upload(ibm_ctx* c, T* dst, const std::vector<T>& src) {
  HIPCHK(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  (void)c;
  return IBM_OK;
}

static int make_twiddles(ibm_ctx* c, FFTPlan* P) {
  std::vector<double2> tw(P->n);
  std::vector<float2> tw32(P->n);
  for (int k = 0; k < P->n; ++k) {
    const long double a = 2.0L * 3.14159265358979323846264338327950288L * k / P->n;
    tw[k] = make_double2((double)cosl(a), (double)(-sinl(a)));
    tw32[k] = make_float2((float)cosl(a), (float)(-sinl(a)));
  }
  double2* d = nullptr;
  float2* d32 = nullptr;
  int rc = dalloc(c, &d, P->n);
  if (rc) return rc;
  rc = dalloc(c, &d32, P->n);
  if (rc) return rc;
  rc = upload(c, d, tw);
  if (rc) return rc;
  rc = upload(c, d32, tw32);
  if (rc) return rc;
  P->tw = d;
  P->tw32 = d32;
  return IBM_OK;
}

// Thomas factorisation tables of the line solves for one beta (host FP64).
static int build_tables(ibm_ctx* c, double beta) {
  if (beta == c->tab_beta) return IBM_OK;
  const int nx = c->nx, nz = c->nz, ny = c->ny;
  std::vector<double> h;
  auto cyclic = [&](int n, double hsp, CyclicTab* t, std::vector<double>& out) {
    const double r = beta / (hsp * hsp);
    const double a = -r, cc = -r, b = 1.0 + 2.0 * r;
    const double gam = -b;
    std::vector<double> cp(n), inv(n), W(n), Z(n), zp(n);
    const double t00 = b - gam;
    const double tnn = b - cc * a / gam;  // corner product A[n-1][0] A[0][n-1]
    inv[0] = 1.0 / t00;
    cp[0] = cc * inv[0];
    for (int i = 1; i < n; ++i) {
      const double bi = (i == n - 1) ? tnn : b;
      inv[i] = 1.0 / (bi - a * cp[i - 1]);
      cp[i] = (i == n - 1) ? 0.0 : cc * inv[i];
    }
    W[0] = 1.0;
    for (int i = 1; i < n; ++i) W[i] = -W[i - 1] * cp[i - 1];
    for (int i = 0; i < n; ++i) {
      const double ui = (i == 0) ? gam : (i == n - 1 ? cc : 0.0);
      zp[i] = (ui - (i ? a * zp[i - 1] : 0.0)) * inv[i];
    }
    Z[n - 1] = zp[n - 1];
    for (int i = n - 2; i >= 0; --i) Z[i] = zp[i] - cp[i] * Z[i + 1];
    t->a = a;
    t->b = b;
    t->c = cc;
    t->ratio = a / gam;
    t->fden_inv = 1.0 / (1.0 + Z[0] + t->ratio * Z[n - 1]);
    for (auto* v : {&cp, &inv, &W, &Z}) out.insert(out.end(), v->begin(), v->end());
  };
  // v: the interior faces j = 1..ny-1 and, as an identity row, the top wall
  // face j = ny (its right-hand side is 0), so that v lines have ny rows like
  // u and w and take the same segmentation
  auto ysys = [&](bool isv, std::vector<double>& out, YTab* t) {
    const int n = ny;
    const int nreal = isv ? ny - 1 : ny;
    std::vector<double> A(n), B(n), C(n), cp(n), inv(n);
    for (int r = 0; r < n; ++r) {
      if (r >= nreal) {
        A[r] = 0.0;
        B[r] = 1.0;
        C[r] = 0.0;
        continue;
      }
      double lo, hi;
      if (isv) {
        const int j = r + 1;
        lo = beta / (c->dy[j - 1] * c->dyc[j]);
        hi = beta / (c->dy[j] * c->dyc[j]);
      } else {
        lo = beta / (c->dyc[r] * c->dy[r]);
        hi = beta / (c->dyc[r + 1] * c->dy[r]);
      }
      A[r] = (r > 0) ? -lo : 0.0;
      C[r] = (r < nreal - 1) ? -hi : 0.0;
      B[r] = 1.0 + (lo + hi);
    }
    for (int r = 0; r < n; ++r) {
      inv[r] = 1.0 / (B[r] - (r ? A[r] * cp[r - 1] : 0.0));
      cp[r] = C[r] * inv[r];
    }
    t->n = n;
    t->j0 = isv ? 1 : 0;
    for (auto* v : {&A, &B, &C, &cp, &inv}) out.insert(out.end(), v->begin(), v->end());
  };
  // elimination tables of the partitioned solve for mask-free segments:
  // [0] 1/pivot, [1] c~ (forward), [2] a^ and [3] c^ (responses of every
  // interior row to the left and right separators), [4] the row's
  // sub-diagonal
  auto segtab = [&](int n, bool cyc, int lmax, const double* A, const double* B, const double* C,
                    std::vector<double>& out) {
    int P, L, r;
    line_plan(n, cyc, lmax, &P, &L, &r);
    std::vector<double> t(LINE_NTAB * (size_t)P * LINE_TLD, 0.0);
    for (int s = 0; s < P; ++s) {
      const int lo = s * L + std::min(s, r);
      const int m = L + (s < r ? 1 : 0) - 1;
      double at = 0, ct = 0;
      std::vector<double> va(m), vc(m);
      for (int e = 0; e < m; ++e) {
        const int i = lo + e;
        const double inv = 1.0 / (B[i] - A[i] * ct);
        at = (e == 0) ? A[i] * inv : -A[i] * at * inv;
        ct = C[i] * inv;
        t[(0 * P + s) * LINE_TLD + e] = inv;
        t[(1 * P + s) * LINE_TLD + e] = ct;
        t[(4 * P + s) * LINE_TLD + e] = A[i];
        va[e] = at;
        vc[e] = ct;
      }
      double ah = 0, ch = 0;
      for (int e = m - 1; e >= 0; --e) {
        if (e == m - 1) {
          ah = va[e];
          ch = vc[e];
        } else {
          ah = va[e] - vc[e] * ah;
          ch = -vc[e] * ch;
        }
        t[(2 * P + s) * LINE_TLD + e] = ah;
        t[(3 * P + s) * LINE_TLD + e] = ch;
      }
    }
    out.insert(out.end(), t.begin(), t.end());
  };
  auto constseg = [&](int n, int lmax, const CyclicTab& t, std::vector<double>& out) {
    std::vector<double> A(n, t.a), B(n, t.b), C(n, t.c);
    segtab(n, true, lmax, A.data(), B.data(), C.data(), out);
  };
  std::vector<double> hx, hz, hy0, hy1, sx, sz, sy0, sy1;
  cyclic(nx, c->g.dx, &c->ctx_x, hx);
  cyclic(nz, c->g.dz, &c->ctx_z, hz);
  ysys(false, hy0, &c->yt[0]);
  ysys(true, hy1, &c->yt[1]);
  constseg(nx, LINE_LMAX, c->ctx_x, sx);
  constseg(nz, z_seg_len(nz, nx, c->fp32), c->ctx_z, sz);
  for (int q = 0; q < 2; ++q) {
    const int n = c->yt[q].n;
    const std::vector<double>& hy = q ? hy1 : hy0;
    segtab(n, false, wall_seg_len(n, nx, c->fp32), hy.data(), hy.data() + n, hy.data() + 2 * n,
           q ? sy1 : sy0);
  }
  for (auto* v : {&hx, &hz, &hy0, &hy1, &sx, &sz, &sy0, &sy1}) h.insert(h.end(), v->begin(), v->end());
  if ((int64_t)h.size() > c->tabcap) {
    g_last_error = "line-solve tables exceed their buffer";
    return IBM_EINVAL;
  }
  // kernels already enqueued read the previous tables: the new ones are
  // copied in stream order, after them, from a pinned staging slot that is
  // rewritten only once its previous copy has completed (the host waits only
  // if the stream is four table changes behind)
  const int ks = c->tab_stage;
  c->tab_stage = (ks + 1) % ibm_ctx::NTSTAGE;
  if (c->tab_used[ks]) HIPCHK(hipEventSynchronize(c->tab_ev[ks]));
  std::memcpy(c->tab_host[ks], h.data(), h.size() * sizeof(double));
  HIPCHK(hipMemcpyAsync(c->tabmem, c->tab_host[ks], h.size() * sizeof(double),
                        hipMemcpyHostToDevice, c->stream));
  if (c->fp32) {  // the same tables rounded to FP32, at the same offsets
    for (size_t q = 0; q < h.size(); ++q) c->tab_host32[ks][q] = (float)h[q];
    HIPCHK(hipMemcpyAsync(c->tabmem32, c->tab_host32[ks], h.size() * sizeof(float),
                          hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(hipEventRecord(c->tab_ev[ks], c->stream));
  c->tab_used[ks] = true;
  int64_t off = 0;
  auto take = [&](int n) {
    const int64_t o = off;
    off += n;
    return o;
  };
  auto d64 = [&](int64_t o) { return (const double*)(c->tabmem + o); };
  auto d32 = [&](int64_t o) { return c->tabmem32 ? (const float*)(c->tabmem32 + o) : nullptr; };
  c->ctx_x.cp = d64(take(nx)); c->ctx_x.inv = d64(take(nx));
  c->ctx_x.W = d64(take(nx)); c->ctx_x.Z = d64(take(nx));
  c->ctx_z.cp = d64(take(nz)); c->ctx_z.inv = d64(take(nz));
  c->ctx_z.W = d64(take(nz)); c->ctx_z.Z = d64(take(nz));
  for (int q = 0; q < 2; ++q) {
    const int n = c->yt[q].n;
    const int64_t oa = take(n), ob = take(n), oc = take(n);
    c->yt[q].a = d64(oa); c->yt[q].b = d64(ob); c->yt[q].c = d64(oc);
    c->yt[q].a32 = d32(oa); c->yt[q].b32 = d32(ob); c->yt[q].c32 = d32(oc);
    c->yt[q].cp = d64(take(n)); c->yt[q].inv = d64(take(n));
  }
  const int64_t ox = take((int)sx.size()), oz = take((int)sz.size());
  const int64_t oy0 = take((int)sy0.size()), oy1 = take((int)sy1.size());
  c->ctx_x.seg = d64(ox); c->ctx_x.seg32 = d32(ox);
  c->ctx_z.seg = d64(oz); c->ctx_z.seg32 = d32(oz);
  c->yt[0].seg = d64(oy0); c->yt[0].seg32 = d32(oy0);
  c->yt[1].seg = d64(oy1); c->yt[1].seg32 = d32(oy1);
  c->tab_beta = beta;
  return IBM_OK;
}

static void free_all(ibm_ctx* c) {
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->hslots) (void)hipHostFree(c->hslots);
  c->hslots = nullptr;
  for (int k = 0; k < ibm_ctx::NTSTAGE; ++k) {
    if (c->tab_host[k]) (void)hipHostFree(c->tab_host[k]);
    if (c->tab_host32[k]) (void)hipHostFree(c->tab_host32[k]);
    if (c->tab_ev[k]) (void)hipEventDestroy(c->tab_ev[k]);
    c->tab_host[k] = nullptr;
    c->tab_host32[k] = nullptr;
    c->tab_ev[k] = nullptr;
  }
  for (auto& e : c->slot_ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& r : c->prof.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->prof.pool) (void)hipEventDestroy(e);
}

extern "C" {

const char* ibm_strerror(int code) {
  switch (code) {
    case IBM_OK: return "ok";
    case IBM_EINVAL: return g_last_error.empty() ? "invalid argument" : g_last_error.c_str();
    case IBM_ENOMEM: return g_last_error.empty() ? "out of device memory" : g_last_error.c_str();
    case IBM_EHIP: return g_last_error.empty() ? "HIP runtime error" : g_last_error.c_str();
    case IBM_ECAPACITY: return "forcing-node or boundary-cell list overflowed its capacity";
    case IBM_ENONFINITE: return "non-finite value in a reduction";
    case IBM_ECFL: return "a body vertex moves more than half the local grid spacing in one step";
    case IBM_ECOMPAT: return "Poisson right-hand side fails the compatibility condition "
                             "(|sum rhs dV| > 1e-12 sum |rhs| dV)";
    case IBM_EGEOM: return "geometry limit: body too large for the periodic box, probe leaving "
                           "the channel, or probe stencil containing its own node";
    default: return "unknown error";
  }
}

#define FAIL(code, msg)     \
  do {                      \
    g_last_error = (msg);   \
    return (code);          \
  } while (0)

int ibm_create(const ibm_grid* gr, const ibm_opts* o, void* stream, ibm_ctx** out) {
  if (!gr || !o || !out) FAIL(IBM_EINVAL, "null argument");
  *out = nullptr;
  if (gr->nx < 8 || gr->nz < 8 || gr->ny < 3) FAIL(IBM_EINVAL, "grid too small (nx, nz >= 8, ny >= 3)");
  if (!gr->y_faces) FAIL(IBM_EINVAL, "y_faces is NULL");
  if (!(gr->lx > 0) || !(gr->lz > 0) || !(o->re > 0)) FAIL(IBM_EINVAL, "lx, lz and re must be > 0");
  if (o->precision != IBM_FP64 && o->precision != IBM_MIXED) FAIL(IBM_EINVAL, "unknown precision");
  if (o->refine_max < 0 || o->refine_max > 16 || o->refine_tol < 0 || !(o->refine_tol == o->refine_tol))
    FAIL(IBM_EINVAL, "refine_max must be 0..16 and refine_tol >= 0");
  if (o->mixed_poisson != IBM_POISSON_FP64 && o->mixed_poisson != IBM_POISSON_REFINED)
    FAIL(IBM_EINVAL, "unknown mixed_poisson");
  if (gr->ny > 8192) FAIL(IBM_EINVAL, "ny above 8192");
  if (gr->nx > 1024 || gr->nz > 1024) FAIL(IBM_EINVAL, "nx and nz at most 1024");
  if (o->scheme != IBM_RK2CN && o->scheme != IBM_AB2CN) FAIL(IBM_EINVAL, "unknown scheme");
  if (o->use_q < IBM_Q_NONE || o->use_q > IBM_Q_ENERGY) FAIL(IBM_EINVAL, "unknown use_q");
  for (int j = 0; j < gr->ny; ++j)
    if (!(gr->y_faces[j + 1] > gr->y_faces[j])) FAIL(IBM_EINVAL, "y_faces not strictly increasing");
  ibm_ctx* c = new ibm_ctx();
  int rc = IBM_OK;
#define TRY(x)                 \
  do {                         \
    rc = (x);                  \
    if (rc) {                  \
      free_all(c);             \
      delete c;                \
      return rc;               \
    }                          \
  } while (0)
  if (hipGetDevice(&c->dev) != hipSuccess) {
    delete c;
    FAIL(IBM_EHIP, "no HIP device");
  }
  c->stream = (hipStream_t)stream;
  c->nx = gr->nx;
  c->ny = gr->ny;
  c->nz = gr->nz;
  c->lx = gr->lx;
  c->lz = gr->lz;
  c->opts = *o;
  c->fp32 = (o->precision == IBM_MIXED) ? 1 : 0;
  c->pfp32 = (c->fp32 && o->mixed_poisson == IBM_POISSON_REFINED) ? 1 : 0;
  c->es = c->fp32 ? sizeof(float) : sizeof(double);
  c->nref = o->refine_max > 0 ? o->refine_max : 3;
  c->rtol = o->refine_tol > 0 ? o->refine_tol : 1e-11;
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  if (!plan_fft(nx, &c->px) || !plan_fft(nz, &c->pz)) {
    delete c;
    FAIL(IBM_EINVAL, "nx and nz must factor into 2, 3, 5 and 7");
  }
  c->ncell = (int64_t)nx * ny * nz;
  c->nvface = (int64_t)nx * (ny + 1) * nz;
  // grid metrics (same operations as any other implementation of the grid)
  c->yf.assign(gr->y_faces, gr->y_faces + ny + 1);
  c->yc.resize(ny);
  c->dy.resize(ny);
  c->dyc.resize(ny + 1);
  for (int j = 0; j < ny; ++j) {
    c->yc[j] = (c->yf[j] + c->yf[j + 1]) * 0.5;
    c->dy[j] = c->yf[j + 1] - c->yf[j];
  }
  c->dyc[0] = c->yc[0] - c->yf[0];
  for (int j = 1; j < ny; ++j) c->dyc[j] = c->yc[j] - c->yc[j - 1];
  c->dyc[ny] = c->yf[ny] - c->yc[ny - 1];
  c->extuw.push_back(c->yf[0]);
  c->extuw.insert(c->extuw.end(), c->yc.begin(), c->yc.end());
  c->extuw.push_back(c->yf[ny]);
  GridView& g = c->g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nxh = nx / 2 + 1;
  g.lx = c->lx;
  g.lz = c->lz;
  g.dx = c->lx / nx;
  g.dz = c->lz / nz;
  double dm = std::max(g.dx, g.dz);
  for (double v : c->dyc) dm = std::max(dm, v);
  for (double v : c->dy) dm = std::max(dm, v);
  g.dmax = dm;
  double *dyf, *dyc_, *ddy, *ddyc, *dext;
  TRY(dalloc(c, &dyf, ny + 1));
  TRY(dalloc(c, &dyc_, ny));
  TRY(dalloc(c, &ddy, ny));
  TRY(dalloc(c, &ddyc, ny + 1));
  TRY(dalloc(c, &dext, ny + 2));
  TRY(upload(c, dyf, c->yf));
  TRY(upload(c, dyc_, c->yc));
  TRY(upload(c, ddy, c->dy));
  TRY(upload(c, ddyc, c->dyc));
  TRY(upload(c, dext, c->extuw));
  g.yf = dyf;
  g.yc = dyc_;
  g.dy = ddy;
  g.dyc = ddyc;
  g.extuw = dext;
  {
    std::vector<double> idy(ny), idyc(ny + 1), fw0(ny + 1, 0.0), fw1(ny + 1, 0.0);
    for (int j = 0; j < ny; ++j) idy[j] = 1.0 / c->dy[j];
    for (int j = 0; j <= ny; ++j) idyc[j] = 1.0 / c->dyc[j];
    for (int f = 1; f < ny; ++f) {
      const double s = c->dy[f - 1] + c->dy[f];
      fw0[f] = c->dy[f] / s;
      fw1[f] = c->dy[f - 1] / s;
    }
    double *a, *b, *d0, *d1;
    TRY(dalloc(c, &a, ny));
    TRY(dalloc(c, &b, ny + 1));
    TRY(dalloc(c, &d0, ny + 1));
    TRY(dalloc(c, &d1, ny + 1));
    TRY(upload(c, a, idy));
    TRY(upload(c, b, idyc));
    TRY(upload(c, d0, fw0));
    TRY(upload(c, d1, fw1));
    g.idy = a;
    g.idyc = b;
    g.fw0 = d0;
    g.fw1 = d1;
    g.idx = 1.0 / g.dx;
    g.idz = 1.0 / g.dz;
  }

  // tag buffers
  TagBuffers& tb = c->tb;
  tb.cap = o->force_cap > 0 ? o->force_cap : std::max<int64_t>(65536, c->ncell / 16);
  int64_t maxw = 0;
  for (int q = 0; q < 3; ++q) {
    const int64_t nn = (q == 1) ? c->nvface : c->ncell;
    tb.nwords[q] = (nn + 31) / 32;
    maxw = std::max(maxw, tb.nwords[q]);
    TRY(dalloc(c, &tb.mask[q], tb.nwords[q]));
    TRY(dalloc(c, &tb.best_d[q], nn));
    TRY(dalloc(c, &tb.best_t[q], nn));
    TRY(dalloc(c, &tb.idx[q], tb.cap));
    TRY(dalloc(c, &tb.tri[q], tb.cap));
  }
  tb.nwords_cb = (c->ncell + 31) / 32;
  TRY(dalloc(c, &tb.cb_mask, tb.nwords_cb));
  TRY(dalloc(c, &tb.cb, tb.cap));
  TRY(dalloc(c, &tb.count, 4));
  tb.bsum_stride = maxw / 1024 + 2;  // >= blocks of 1024 mask words of any list
  TRY(dalloc(c, &tb.block_sums, 3 * tb.bsum_stride));
  TRY(dalloc(c, &c->force_vals, 3 * tb.cap));
  TRY(dalloc(c, &c->dslots, (int64_t)ibm_ctx::NSLOT * ibm_ctx::MAXB));
  if (hipHostMalloc((void**)&c->hslots, sizeof(BodyDev) * ibm_ctx::NSLOT * ibm_ctx::MAXB) != hipSuccess) {
    c->hslots = nullptr;
    TRY(IBM_ENOMEM);
  }
  for (int q = 0; q < ibm_ctx::NSLOT; ++q)
    if (hipEventCreateWithFlags(&c->slot_ev[q], hipEventDisableTiming) != hipSuccess) TRY(IBM_EHIP);

  for (int q = 0; q < 3; ++q) {
    const int64_t nn = (q == 1) ? c->nvface : c->ncell;
    TRY(dalloc_bytes(c, &c->R[q], nn, c->es));
    TRY(dalloc_bytes(c, &c->H[q], nn, c->es));
  }
  TRY(dalloc_bytes(c, &c->sa, c->nvface, c->es));
  TRY(dalloc_bytes(c, &c->sc, c->nvface, c->es));
  TRY(dalloc(c, &c->phi, c->ncell));
  const int64_t nspec = (int64_t)ny * nz * spec_ld(g.nxh, c->pfp32);
  TRY(dalloc_bytes(c, &c->spec, nspec, c->pfp32 ? 2 * sizeof(float) : 2 * sizeof(double)));
  if (c->pfp32) {
    TRY(dalloc_bytes(c, &c->spec64, (int64_t)ny * nz * spec_ld(g.nxh, false), 2 * sizeof(double)));
    TRY(dalloc(c, &c->rhs_keep, c->ncell));
    TRY(dalloc(c, &c->rmax, c->nref + 2));
    TRY(dalloc(c, &c->zm, ny));
    TRY(dalloc(c, &c->msum, c->nref + 2));
    // per-block partials of the x passes (at least one x-row per block)
    TRY(dalloc(c, &c->psum, (int64_t)ny * nz));
  }
  TRY(dalloc(c, &c->rstats, IBM_REFINE_STATS));
  TRY(dalloc(c, &c->partial, 5 * 512));  // block partials of the mass sums
  TRY(dalloc(c, &c->qf, 2));              // q_F, or (c0, c1) of the energy shape
  TRY(dalloc(c, &c->diag, 4));
  TRY(dalloc(c, &c->flags, 1));
  {
    int P, L, r, segs = 0;
    line_plan(nx, true, &P, &L, &r);
    segs += P;
    line_plan(nz, true, z_seg_len(nz, nx, c->fp32), &P, &L, &r);
    segs += P;
    line_plan(ny, false, wall_seg_len(ny, nx, c->fp32), &P, &L, &r);
    segs += 2 * P;
    c->tabcap = 4 * (int64_t)(nx + nz) + 10 * (int64_t)ny + LINE_NTAB * (int64_t)segs * LINE_TLD;
    TRY(dalloc(c, &c->tabmem, c->tabcap));
    if (c->fp32) TRY(dalloc(c, &c->tabmem32, c->tabcap));
    for (int k = 0; k < ibm_ctx::NTSTAGE; ++k) {
      if (hipHostMalloc((void**)&c->tab_host[k], sizeof(double) * c->tabcap) != hipSuccess) {
        c->tab_host[k] = nullptr;
        TRY(IBM_ENOMEM);
      }
      if (c->fp32 &&
          hipHostMalloc((void**)&c->tab_host32[k], sizeof(float) * c->tabcap) != hipSuccess) {
        c->tab_host32[k] = nullptr;
        TRY(IBM_ENOMEM);
      }
      if (hipEventCreateWithFlags(&c->tab_ev[k], hipEventDisableTiming) != hipSuccess) TRY(IBM_EHIP);
    }
  }

  // Poisson tables
  TRY(make_twiddles(c, &c->px));
  TRY(make_twiddles(c, &c->pz));
  {
    std::vector<double> lx(g.nxh), lz(nz), lo(ny, 0.0), hi(ny, 0.0);
    const double pi = 3.14159265358979323846;
    for (int p = 0; p < g.nxh; ++p) {
      const double s = std::sin(pi * p / nx);
      lx[p] = -(4.0 / (g.dx * g.dx)) * s * s;
    }
    for (int m = 0; m < nz; ++m) {
      const double s = std::sin(pi * m / nz);
      lz[m] = -(4.0 / (g.dz * g.dz)) * s * s;
    }
    for (int j = 1; j < ny; ++j) lo[j] = 1.0 / (c->dyc[j] * c->dy[j]);
    for (int j = 0; j + 1 < ny; ++j) hi[j] = 1.0 / (c->dyc[j + 1] * c->dy[j]);
    TRY(dalloc(c, &c->lamx, g.nxh));
    TRY(dalloc(c, &c->lamz, nz));
    TRY(dalloc(c, &c->ylo, ny));
    TRY(dalloc(c, &c->yhi, ny));
    TRY(upload(c, c->lamx, lx));
    TRY(upload(c, c->lamz, lz));
    TRY(upload(c, c->ylo, lo));
    TRY(upload(c, c->yhi, hi));
    c->sum_dy = 0;
    for (double v : c->dy) c->sum_dy += v;
    c->vtot = g.dx * g.dz * (double)nx * (double)nz * c->sum_dy;
  }
  // initial state of the tag scratch: best keys at +inf, flags clear
  for (int q = 0; q < 3; ++q) {
    const int64_t nn = (q == 1) ? c->nvface : c->ncell;
    launch_fill_u64(nullptr, c->stream, tb.best_d[q], nn, ~0ull);
    launch_fill_i32(nullptr, c->stream, tb.best_t[q], nn, 0x7fffffff);
    launch_fill_u32(nullptr, c->stream, tb.mask[q], tb.nwords[q], 0u);
  }
  launch_fill_u32(nullptr, c->stream, tb.cb_mask, tb.nwords_cb, 0u);
  launch_fill_u32(nullptr, c->stream, c->flags, 1, 0u);
  launch_fill_u64(nullptr, c->stream, reinterpret_cast<u64*>(tb.count), 4, 0ull);
  launch_fill_f64(nullptr, c->stream, c->qf, 2, 0.0);
  launch_fill_f64(nullptr, c->stream, c->rstats, IBM_REFINE_STATS, 0.0);
  if (hipStreamSynchronize(c->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
    free_all(c);
    delete c;
    FAIL(IBM_EHIP, "initialisation kernels failed");
  }
#undef TRY
  *out = c;
  return IBM_OK;
}

void ibm_destroy(ibm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

int ibm_set_stream(ibm_ctx* c, void* stream) {
  if (!c) FAIL(IBM_EINVAL, "null context");
  c->stream = (hipStream_t)stream;
  return IBM_OK;
}

static int launch_status() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) FAIL(IBM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return IBM_OK;
}

int ibm_body_rigid(ibm_ctx* c, const double* x0, int32_t nv, const double* coef, double* xyz,
                   double* vel) {
  if (!c || !coef || nv < 0 || (nv > 0 && (!x0 || !xyz || !vel))) FAIL(IBM_EINVAL, "ibm_body_rigid: bad argument");
  launch_body_rigid(&c->prof, c->stream, x0, nv, coef, xyz, vel);
  return launch_status();
}

int ibm_body_rigid_dev(ibm_ctx* c, const double* x0, int32_t nv, const double* coef,
                       double* xyz, double* vel) {
  if (!c || !coef || nv < 0 || (nv > 0 && (!x0 || !xyz || !vel)))
    FAIL(IBM_EINVAL, "ibm_body_rigid_dev: bad argument");
  launch_body_dev(&c->prof, c->stream, 0, x0, nv, coef, xyz, vel);
  return launch_status();
}

int ibm_rigid_advance(ibm_ctx* c, int32_t nb, double* state, const double* props,
                      const double* loads, double dt, double* coef) {
  if (!c || nb < 0 || (nb > 0 && (!state || !props || !loads || !coef)) || !(dt > 0))
    FAIL(IBM_EINVAL, "ibm_rigid_advance: bad argument");
  launch_rigid_advance(&c->prof, c->stream, nb, state, props, loads, dt, coef);
  return launch_status();
}

int ibm_body_deform(ibm_ctx* c, const double* data, int32_t nv, const double* coef, double* xyz,
                    double* vel) {
  if (!c || !coef || nv < 0 || (nv > 0 && (!data || !xyz || !vel))) FAIL(IBM_EINVAL, "ibm_body_deform: bad argument");
  launch_body_deform(&c->prof, c->stream, data, nv, coef, xyz, vel);
  return launch_status();
}

static int set_bodies(ibm_ctx* c, const ibm_body* b, int32_t nb) {
  if (nb < 0 || (nb > 0 && !b)) FAIL(IBM_EINVAL, "bad body list");
  if (nb > ibm_ctx::MAXB) FAIL(IBM_EINVAL, "at most 128 bodies per context");
  c->bodies.clear();
  int64_t off = 0;
  for (int i = 0; i < nb; ++i) {
    if (b[i].nt < 0 || b[i].nv < 0 || (b[i].nt > 0 && (!b[i].xyz || !b[i].vel || !b[i].tri)))
      FAIL(IBM_EINVAL, "bad body");
    BodyDev d;
    d.xyz = b[i].xyz;
    d.vel = b[i].vel;
    d.tri = b[i].tri;
    d.nt = b[i].nt;
    d.toff = (int32_t)off;
    off += b[i].nt;
    if (off > INT32_MAX) FAIL(IBM_EINVAL, "too many triangles");
    c->bodies.push_back(d);
  }
  c->ntri = (int)off;
  return IBM_OK;
}

}  // extern "C"

// Body descriptors live in device memory: a small ring of device slots
// filled by stream-ordered copies from pinned host slots.  An unchanged list
// (the usual case from one step to the next) reuses the current slot and
// costs no copy; a pinned slot is rewritten only after its previous copy has
// completed (its event), so no copy ever reads a slot being rewritten.
static int upload_bodies(ibm_ctx* c) {
  const size_t n = c->bodies.size();
  if (n == 0) {
    c->d_bodies = nullptr;
    return IBM_OK;
  }
  if (c->cur_slot >= 0 && c->last_bodies == c->bodies) {
    c->d_bodies = c->dslots + (size_t)c->cur_slot * ibm_ctx::MAXB;
    return IBM_OK;
  }
  const int k = (c->cur_slot + 1) % ibm_ctx::NSLOT;
  if (c->slot_used[k]) HIPCHK(hipEventSynchronize(c->slot_ev[k]));
  std::memcpy(c->hslots + (size_t)k * ibm_ctx::MAXB, c->bodies.data(), n * sizeof(BodyDev));
  HIPCHK(hipMemcpyAsync(c->dslots + (size_t)k * ibm_ctx::MAXB, c->hslots + (size_t)k * ibm_ctx::MAXB,
                        n * sizeof(BodyDev), hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipEventRecord(c->slot_ev[k], c->stream));
  c->slot_used[k] = true;
  c->cur_slot = k;
  c->last_bodies = c->bodies;
  c->d_bodies = c->dslots + (size_t)k * ibm_ctx::MAXB;
  return IBM_OK;
}

extern "C" {

}  // extern "C"

// tagging; dt > 0 also checks the vertex displacement over dt (FLAG_CFL)
static int tag_bodies(ibm_ctx* c, const ibm_body* b, int32_t nb, ibm_tags* out, double dt) {
  int rc = set_bodies(c, b, nb);
  if (rc) return rc;
  rc = upload_bodies(c);
  if (rc) return rc;
  launch_tag(&c->prof, c->stream, c->g, c->d_bodies, (int)c->bodies.size(), c->ntri, c->tb,
             c->flags, dt);
  rc = launch_status();
  if (rc) return rc;
  if (out) {
    for (int q = 0; q < 3; ++q) {
      out->idx[q] = c->tb.idx[q];
      out->tri[q] = c->tb.tri[q];
      out->mask[q] = c->tb.mask[q];
    }
    out->cb = c->tb.cb;
    out->count = c->tb.count;
    out->cb_mask = c->tb.cb_mask;
    out->capacity = c->tb.cap;
  }
  return IBM_OK;
}

extern "C" {

int ibm_tag(ibm_ctx* c, const ibm_body* b, int32_t nb, ibm_tags* out) {
  if (!c) FAIL(IBM_EINVAL, "null context");
  return tag_bodies(c, b, nb, out, 0.0);
}

int ibm_tags_count_host(ibm_ctx* c, int64_t* counts) {
  if (!c || !counts) FAIL(IBM_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(counts, c->tb.count, 4 * sizeof(int64_t), hipMemcpyDeviceToHost));
  return IBM_OK;
}

int ibm_tags_copy(ibm_ctx* c, int32_t list, int64_t* idx_dst, int32_t* tri_dst, int64_t n) {
  if (!c || list < 0 || list > 3 || n < 0 || n > c->tb.cap || (n > 0 && !idx_dst))
    FAIL(IBM_EINVAL, "ibm_tags_copy: bad argument");
  if (n == 0) return IBM_OK;
  const int64_t* src = (list == 3) ? c->tb.cb : c->tb.idx[list];
  HIPCHK(hipMemcpyAsync(idx_dst, src, n * sizeof(int64_t), hipMemcpyDeviceToDevice, c->stream));
  if (tri_dst && list < 3)
    HIPCHK(hipMemcpyAsync(tri_dst, c->tb.tri[list], n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                          c->stream));
  return IBM_OK;
}

int ibm_force(ibm_ctx* c, double* u, double* v, double* w) {
  if (!c || !u || !v || !w) FAIL(IBM_EINVAL, "null argument");
  double* f[3] = {u, v, w};
  launch_force(&c->prof, c->stream, c->g, c->d_bodies, (int)c->bodies.size(), c->tb, f,
               c->force_vals, c->flags);
  return launch_status();
}

static int viscous(ibm_ctx* c, const void* p, const void* const* hprev, void* const* hout,
                   double gamma, double rho, double dt, double* u, double* v, double* w) {
  const double alpha = gamma + rho;
  int rc = build_tables(c, alpha * dt / (2.0 * c->opts.re));
  if (rc) return rc;
  RhsArgs a{};
  a.u = u;
  a.v = v;
  a.w = w;
  a.p = p;
  for (int q = 0; q < 3; ++q) {
    a.hprev[q] = hprev ? hprev[q] : nullptr;
    a.hout[q] = hout ? hout[q] : nullptr;
    a.R[q] = c->R[q];
    a.mask[q] = c->tb.mask[q];
  }
  if (rho != 0.0 && (!a.hprev[0] || !a.hprev[1] || !a.hprev[2]))
    FAIL(IBM_EINVAL, "rho != 0 needs the previous H");
  if ((a.hout[0] || a.hout[1] || a.hout[2]) && !(a.hout[0] && a.hout[1] && a.hout[2]))
    FAIL(IBM_EINVAL, "h_out: all three components or none");
  a.gamma = gamma;
  a.rho = rho;
  a.alpha = alpha;
  a.dt = dt;
  a.re = c->opts.re;
  a.fx = -c->opts.dpdx;
  a.fp32 = c->fp32;
  a.planes = c->rhs_planes;
  launch_rhs(&c->prof, c->stream, c->g, a);
  double* f[3] = {u, v, w};
  for (int q = 0; q < 3; ++q)
    if (c->vf0[q] || c->vkap[q])
      launch_vforce(&c->prof, c->stream, c->g, q, c->R[q], c->fp32, c->tb.mask[q], f[q],
                    c->vf0[q], c->vkap[q], alpha * dt);
  for (int q = 0; q < 3; ++q) {
    launch_adi_x(&c->prof, c->stream, c->g, q, c->R[q], c->tb.mask[q], c->ctx_x, c->sa, c->sc,
                 c->fp32);
    launch_adi_z(&c->prof, c->stream, c->g, q, c->R[q], c->tb.mask[q], c->ctx_z, c->sa, c->sc,
                 c->fp32);
    launch_adi_y(&c->prof, c->stream, c->g, q, c->R[q], f[q], c->tb.mask[q],
                 c->yt[q == 1 ? 1 : 0], c->sa, c->sc, c->fp32);
  }
  return launch_status();
}

int ibm_set_volume_force(ibm_ctx* c, int32_t comp, const double* f0, const double* kappa) {
  if (!c || comp < 0 || comp > 2) FAIL(IBM_EINVAL, "ibm_set_volume_force: bad argument");
  c->vf0[comp] = f0;
  c->vkap[comp] = kappa;
  return IBM_OK;
}

int ibm_viscous(ibm_ctx* c, const void* p, const void* const* h_prev, void* const* h_out,
                double gamma, double rho, double dt, double* u, double* v, double* w) {
  if (!c || !p || !u || !v || !w || !(dt > 0)) FAIL(IBM_EINVAL, "ibm_viscous: bad argument");
  return viscous(c, p, h_prev, h_out, gamma, rho, dt, u, v, w);
}

int ibm_mass_rhs(ibm_ctx* c, const double* u, const double* v, const double* w, const void* p,
                 double alpha_dt, double* rhs, double* qf) {
  if (!c || !u || !v || !w || !rhs || !(alpha_dt > 0)) FAIL(IBM_EINVAL, "ibm_mass_rhs: bad argument");
  if (c->opts.use_q == IBM_Q_ENERGY) {
    if (!p) FAIL(IBM_EINVAL, "ibm_mass_rhs: the energy-conserving shape needs p");
    launch_mass_energy(&c->prof, c->stream, c->g, u, v, w, p, c->fp32, c->tb.cb_mask, c->partial,
                       c->qf, c->flags);
    launch_mass_rhs_energy(&c->prof, c->stream, c->g, u, v, w, p, c->fp32, c->tb.cb_mask, c->qf,
                           1.0 / alpha_dt, rhs);
  } else {
    launch_mass(&c->prof, c->stream, c->g, u, v, w, c->tb.cb, c->tb.count, c->tb.cap, c->vtot,
                c->opts.use_q, c->partial, c->qf, c->flags);
    launch_mass_rhs(&c->prof, c->stream, c->g, u, v, w, c->opts.use_q ? c->tb.cb_mask : nullptr,
                    c->qf, 1.0 / alpha_dt, rhs);
  }
  const size_t nq = (c->opts.use_q == IBM_Q_ENERGY) ? 2 : 1;
  if (qf) HIPCHK(hipMemcpyAsync(qf, c->qf, nq * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return launch_status();
}

static PoissonArgs pargs(ibm_ctx* c) {
  PoissonArgs a{};
  a.px = &c->px;
  a.pz = &c->pz;
  a.lamx = c->lamx;
  a.lamz = c->lamz;
  a.ylo = c->ylo;
  a.yhi = c->yhi;
  a.spec = c->spec;
  a.spec64 = c->spec64;
  a.sum_dy = c->sum_dy;
  a.fp32 = c->pfp32;
  a.refine = c->pfp32;
  a.p_fp32 = c->fp32;
  a.nref = c->nref;
  a.tol = c->rtol;
  a.rhs_keep = c->rhs_keep;
  a.rmax = c->rmax;
  a.stats = c->rstats;
  a.zm = c->zm;
  a.psum = c->psum;
  a.msum = c->msum;
  a.vtot = c->vtot;
  a.flags = c->flags;
  return a;
}

int poisson_solve(ibm_ctx* c, const double* rhs, double* phi) {
  if (!c || !rhs || !phi) FAIL(IBM_EINVAL, "poisson_solve: bad argument");
  launch_compat(&c->prof, c->stream, c->g, rhs, c->partial, c->flags);
  launch_poisson(&c->prof, c->stream, c->g, pargs(c), rhs, nullptr, nullptr, nullptr, nullptr,
                 nullptr, nullptr, 1.0, phi);
  return launch_status();
}

int ibm_noslip_error(ibm_ctx* c, const double* u, const double* v, const double* w,
                     double* eps) {
  if (!c || !u || !v || !w || !eps) FAIL(IBM_EINVAL, "ibm_noslip_error: bad argument");
  const double* f[3] = {u, v, w};
  launch_noslip(&c->prof, c->stream, c->g, c->d_bodies, (int)c->bodies.size(), c->tb, f,
                c->force_vals, c->diag, c->flags);
  int rc = launch_status();
  if (rc) return rc;
  double h[3];
  HIPCHK(hipMemcpyAsync(h, c->diag, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  eps[1] = h[0];
  eps[2] = h[1];
  eps[3] = h[2];
  eps[0] = (h[0] + h[1] + h[2]) / 3.0;
  return IBM_OK;
}

int ibm_divergence(ibm_ctx* c, const double* u, const double* v, const double* w,
                   double* out) {
  if (!c || !u || !v || !w || !out) FAIL(IBM_EINVAL, "ibm_divergence: bad argument");
  launch_divergence(&c->prof, c->stream, c->g, u, v, w,
                    c->opts.use_q ? c->tb.cb_mask : nullptr, c->qf, c->partial, c->diag);
  int rc = launch_status();
  if (rc) return rc;
  double h[2];
  HIPCHK(hipMemcpyAsync(h, c->diag, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(h + 1, c->qf, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  out[0] = h[0];
  out[1] = h[1];
  return IBM_OK;
}

int ibm_loads(ibm_ctx* c, const double* u, const double* v, const double* w, const void* p,
              const int32_t* sides, const double* pole, double* traction, double* loads) {
  if (!c || !u || !v || !w || !p || !sides || !pole || !traction || !loads)
    FAIL(IBM_EINVAL, "ibm_loads: null argument");
  if (c->bodies.empty()) FAIL(IBM_EINVAL, "ibm_loads: no bodies in the last tagging");
  launch_loads(&c->prof, c->stream, c->g, c->d_bodies, (int)c->bodies.size(), c->ntri, u, v, w,
               p, c->fp32, c->tb.cb_mask, sides, pole, c->opts.re, traction, loads);
  return launch_status();
}

int ibm_pressure_cb(ibm_ctx* c, const void* p, double* out, int64_t out_cap) {
  if (!c || !p || (!out && out_cap > 0) || out_cap < 0)
    FAIL(IBM_EINVAL, "ibm_pressure_cb: bad argument");
  launch_pressure_cb(&c->prof, c->stream, c->g, c->d_bodies, (int)c->bodies.size(), c->tb, p,
                     c->fp32, out, out_cap, c->flags);
  return launch_status();
}

int ibm_project(ibm_ctx* c, const double* phi, double alpha_dt, double* u, double* v, double* w,
                void* p) {
  if (!c || !phi || !u || !v || !w || !p) FAIL(IBM_EINVAL, "ibm_project: bad argument");
  launch_project(&c->prof, c->stream, c->g, phi, alpha_dt, c->opts.re, u, v, w, p, c->fp32);
  return launch_status();
}

int ibm_step(ibm_ctx* c, ibm_state* s, const ibm_body* b, int32_t nb, double dt) {
  if (!c || !s || !s->u || !s->v || !s->w || !s->p || !(dt > 0)) FAIL(IBM_EINVAL, "ibm_step: bad argument");
  int rc = tag_bodies(c, b, nb, nullptr, dt);
  if (rc) return rc;
  struct Sub {
    double gamma, rho;
    const void* const* hprev;
    void* const* hout;
  };
  void* H1[3] = {c->H[0], c->H[1], c->H[2]};
  std::vector<Sub> subs;
  if (c->opts.scheme == IBM_RK2CN) {
    subs.push_back({0.5, 0.0, nullptr, H1});
    subs.push_back({1.0, -0.5, H1, nullptr});
  } else {
    if (!s->h[0] || !s->h[1] || !s->h[2]) FAIL(IBM_EINVAL, "AB+CN needs state->h");
    subs.push_back({1.5, -0.5, s->h, s->h});
  }
  double* f[3] = {s->u, s->v, s->w};
  for (const Sub& sb : subs) {
    const double alpha = sb.gamma + sb.rho;
    launch_force(&c->prof, c->stream, c->g, c->d_bodies, (int)c->bodies.size(), c->tb, f,
                 c->force_vals, c->flags);
    rc = viscous(c, s->p, sb.hprev, sb.hout, sb.gamma, sb.rho, dt, s->u, s->v, s->w);
    if (rc) return rc;
    const bool energy = c->opts.use_q == IBM_Q_ENERGY;
    if (energy)
      launch_mass_energy(&c->prof, c->stream, c->g, s->u, s->v, s->w, s->p, c->fp32,
                         c->tb.cb_mask, c->partial, c->qf, c->flags);
    else
      launch_mass(&c->prof, c->stream, c->g, s->u, s->v, s->w, c->tb.cb, c->tb.count, c->tb.cap,
                  c->vtot, c->opts.use_q, c->partial, c->qf, c->flags);
    launch_poisson(&c->prof, c->stream, c->g, pargs(c), nullptr, s->u, s->v, s->w,
                   c->opts.use_q ? c->tb.cb_mask : nullptr, c->qf, energy ? s->p : nullptr,
                   1.0 / (alpha * dt), c->phi);
    launch_project(&c->prof, c->stream, c->g, c->phi, alpha * dt, c->opts.re, s->u, s->v, s->w,
                   s->p, c->fp32);
    rc = launch_status();
    if (rc) return rc;
  }
  return IBM_OK;
}

int ibm_refine_stats(ibm_ctx* c, double* stats, int32_t reset) {
  if (!c || !stats) FAIL(IBM_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(stats, c->rstats, IBM_REFINE_STATS * sizeof(double), hipMemcpyDeviceToHost));
  if (reset) {
    launch_fill_f64(nullptr, c->stream, c->rstats, IBM_REFINE_STATS, 0.0);
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  return IBM_OK;
}

int ibm_check(ibm_ctx* c, uint32_t* flags) {
  if (!c || !flags) FAIL(IBM_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(flags, c->flags, sizeof(uint32_t), hipMemcpyDeviceToHost));
  launch_fill_u32(nullptr, c->stream, c->flags, 1, 0u);
  HIPCHK(hipStreamSynchronize(c->stream));
  return IBM_OK;
}

int ibm_profile(ibm_ctx* c, int32_t enable, const char* filter) {
  if (!c) FAIL(IBM_EINVAL, "null context");
  c->prof.enabled = enable != 0;
  c->prof.filter = filter ? filter : "";
  return IBM_OK;
}

int ibm_profile_read(ibm_ctx* c, char* names, int32_t name_len, int64_t* launches,
                     double* total_ms, int32_t cap) {
  if (!c) FAIL(IBM_EINVAL, "null context");
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<std::string> nm;
  std::vector<int64_t> cnt;
  std::vector<double> tot;
  for (auto& r : c->prof.recs) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    size_t k = 0;
    while (k < nm.size() && nm[k] != r.name) ++k;
    if (k == nm.size()) {
      nm.push_back(r.name);
      cnt.push_back(0);
      tot.push_back(0.0);
    }
    cnt[k] += 1;
    tot[k] += ms;
    c->prof.pool.push_back(r.a);
    c->prof.pool.push_back(r.b);
  }
  c->prof.recs.clear();
  int n = 0;
  for (size_t k = 0; k < nm.size() && n < cap; ++k, ++n) {
    if (names && name_len > 0) {
      std::strncpy(names + (size_t)n * name_len, nm[k].c_str(), name_len - 1);
      names[(size_t)n * name_len + name_len - 1] = 0;
    }
    if (launches) launches[n] = cnt[k];
    if (total_ms) total_ms[n] = tot[k];
  }
  return n;
}

}  // extern "C"

// ------------------------------------------------------------ batch support
namespace ibm {

hipStream_t ctx_stream(ibm_ctx* c) { return c->stream; }
Prof* ctx_prof(ibm_ctx* c) { return &c->prof; }

// Everything a time step may need to do outside stream order, done ahead of
// a graph capture: the body descriptors in device memory and the line-solve
// tables of the scheme's beta for this dt (the sub-stages of both schemes
// share one alpha).
int ctx_prepare(ibm_ctx* c, const ibm_body* b, int32_t nb, double dt) {
  int rc = set_bodies(c, b, nb);
  if (rc) return rc;
  rc = upload_bodies(c);
  if (rc) return rc;
  const double alpha = (c->opts.scheme == IBM_RK2CN) ? 1.0 + -0.5 : 1.5 + -0.5;
  rc = build_tables(c, alpha * dt / (2.0 * c->opts.re));
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  return IBM_OK;
}

int ctx_fail(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

void ctx_set_rhs_planes(ibm_ctx* c, int planes) { c->rhs_planes = planes; }

// element counts of the state arrays and their element sizes: u, w and p
// have ncell values, v nvface; u, v, w are FP64; p and the AB2 H arrays are
// pbytes wide (8, or 4 in the mixed form)
void ctx_state_layout(ibm_ctx* c, int64_t* ncell, int64_t* nvface, int* pbytes) {
  *ncell = c->ncell;
  *nvface = c->nvface;
  *pbytes = (int)c->es;
}

}  // namespace ibm
