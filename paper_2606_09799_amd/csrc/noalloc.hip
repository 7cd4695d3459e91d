// Context-free Poisson solve for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the direct solve of poisson_solve (paper Eq. elliptic /
// elliptic_mod: real FFT in x, complex FFT in z, tridiagonal solves in y per
// mode, the (0,0) mode gauged), FP64, with every table and the spectrum in
// one file-scope device array instead of a context's workspace.
//
// The array is `scratch` below (IBM_STATIC_SCRATCH_BYTES, a fixed size; each
// device the library runs on holds it until the process ends).  Its device
// address is taken once per device with hipGetSymbolAddress, with that
// device current, and only that address is used from the host.  Per call:
//   - the y faces go to the device as kernel arguments (chunks of a fixed
//     struct, so a captured launch keeps its own copy; no host buffer has to
//     outlive the call, no copy engine is involved);
//   - one setup kernel derives every grid table from them (the operations of
//     the context's host-side set-up, in the same order, and the transform
//     twiddles and periodic eigenvalues from sincospi);
//   - the solve runs the kernels of the context path on these tables.
// Calls that overlap on one device share the array and race; calls on one
// stream are ordered.  The flag word in the array is cleared by each call
// (a fill kernel, not a memset) and is not reported: this entry point has no
// context to read flags from.
#include "ibm.h"

#include <cmath>
#include <mutex>

#include "internal.h"

namespace ibm {

static __device__ __align__(256) unsigned char scratch[IBM_STATIC_SCRATCH_BYTES];

constexpr int FACES_CHUNK = 448;  // y faces per store launch (3.6 KB of kernel arguments)
struct FaceChunk {
  int first, count;
  double v[FACES_CHUNK];
};

__global__ void k_store_faces(FaceChunk c, double* yf) {
  for (int q = threadIdx.x; q < c.count; q += blockDim.x) yf[c.first + q] = c.v[q];
}

// Offsets (in doubles) of the tables inside the scratch array.
struct StaticLayout {
  int64_t yf, yc, dy, dyc, extuw, idy, idyc, fw0, fw1, ylo, yhi, lamx, lamz, twx, twz, flags, spec;
  int64_t bytes;
};

static StaticLayout static_layout(int nx, int ny, int nz) {
  StaticLayout L{};
  int64_t off = 0;
  auto take = [&](int64_t n) {
    const int64_t o = off;
    off += (n + 31) / 32 * 32;  // 256-byte pieces
    return o;
  };
  const int nxh = nx / 2 + 1;
  L.yf = take(ny + 1);
  L.yc = take(ny);
  L.dy = take(ny);
  L.dyc = take(ny + 1);
  L.extuw = take(ny + 2);
  L.idy = take(ny);
  L.idyc = take(ny + 1);
  L.fw0 = take(ny + 1);
  L.fw1 = take(ny + 1);
  L.ylo = take(ny);
  L.yhi = take(ny);
  L.lamx = take(nxh);
  L.lamz = take(nz);
  L.twx = take(2 * (int64_t)nx);
  L.twz = take(2 * (int64_t)nz);
  L.flags = take(1);
  L.spec = take(2 * (int64_t)ny * nz * spec_ld(nxh, false));
  L.bytes = off * (int64_t)sizeof(double);
  return L;
}

// every table of the grid from the faces already in yf (one block)
__global__ void k_static_tables(double* base, StaticLayout L, int nx, int ny, int nz, double dx,
                                double dz) {
  double* yf = base + L.yf;
  double* yc = base + L.yc;
  double* dy = base + L.dy;
  double* dyc = base + L.dyc;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int j = t; j < ny; j += nt) {
    yc[j] = (yf[j] + yf[j + 1]) * 0.5;
    dy[j] = yf[j + 1] - yf[j];
  }
  __syncthreads();
  for (int j = t; j <= ny; j += nt) {
    const double d = (j == 0) ? yc[0] - yf[0] : (j == ny ? yf[ny] - yc[ny - 1] : yc[j] - yc[j - 1]);
    dyc[j] = d;
    base[L.idyc + j] = 1.0 / d;
    double w0 = 0.0, w1 = 0.0;
    if (j >= 1 && j < ny) {
      const double s = dy[j - 1] + dy[j];
      w0 = dy[j] / s;
      w1 = dy[j - 1] / s;
    }
    base[L.fw0 + j] = w0;
    base[L.fw1 + j] = w1;
  }
  for (int j = t; j < ny + 2; j += nt)
    base[L.extuw + j] = (j == 0) ? yf[0] : (j == ny + 1 ? yf[ny] : yc[j - 1]);
  for (int j = t; j < ny; j += nt) base[L.idy + j] = 1.0 / dy[j];
  __syncthreads();
  for (int j = t; j < ny; j += nt) {
    base[L.ylo + j] = (j >= 1) ? 1.0 / (dyc[j] * dy[j]) : 0.0;
    base[L.yhi + j] = (j + 1 < ny) ? 1.0 / (dyc[j + 1] * dy[j]) : 0.0;
  }
  const int nxh = nx / 2 + 1;
  for (int p = t; p < nxh; p += nt) {
    const double s = sinpi((double)p / nx);
    base[L.lamx + p] = -(4.0 / (dx * dx)) * s * s;
  }
  for (int m = t; m < nz; m += nt) {
    const double s = sinpi((double)m / nz);
    base[L.lamz + m] = -(4.0 / (dz * dz)) * s * s;
  }
  for (int k = t; k < nx; k += nt) {
    double sn, cs;
    sincospi(2.0 * k / nx, &sn, &cs);
    base[L.twx + 2 * k] = cs;
    base[L.twx + 2 * k + 1] = -sn;
  }
  for (int k = t; k < nz; k += nt) {
    double sn, cs;
    sincospi(2.0 * k / nz, &sn, &cs);
    base[L.twz + 2 * k] = cs;
    base[L.twz + 2 * k + 1] = -sn;
  }
  if (t == 0) reinterpret_cast<uint32_t*>(base + L.flags)[0] = 0u;
}

// the scratch array's device address on each device (taken once per device,
// with that device current)
constexpr int MAX_DEVICES = 64;
static void* g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mu;

static int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return IBM_EHIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return IBM_OK;
}

int ctx_fail(int code, const char* msg);

}  // namespace ibm

using namespace ibm;

extern "C" int poisson_solve_static(const ibm_grid* gr, const double* rhs, double* phi,
                                    void* stream) {
  if (!gr || !rhs || !phi || !gr->y_faces)
    return ctx_fail(IBM_EINVAL, "poisson_solve_static: null argument");
  const int nx = gr->nx, ny = gr->ny, nz = gr->nz;
  if (nx < 8 || nz < 8 || ny < 3 || nx > 1024 || nz > 1024 || ny > 8192 || !(gr->lx > 0) ||
      !(gr->lz > 0))
    return ctx_fail(IBM_EINVAL, "poisson_solve_static: bad grid");
  for (int j = 0; j < ny; ++j)
    if (!(gr->y_faces[j + 1] > gr->y_faces[j]))
      return ctx_fail(IBM_EINVAL, "poisson_solve_static: y_faces not strictly increasing");
  FFTPlan px{}, pz{};
  if (!plan_fft(nx, &px) || !plan_fft(nz, &pz))
    return ctx_fail(IBM_EINVAL, "poisson_solve_static: nx and nz must factor into 2, 3, 5, 7");
  const StaticLayout L = static_layout(nx, ny, nz);
  if (L.bytes > (int64_t)IBM_STATIC_SCRATCH_BYTES)
    return ctx_fail(IBM_EINVAL, "poisson_solve_static: the grid needs more than the "
                                "IBM_STATIC_SCRATCH_BYTES of the static workspace");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
    return ctx_fail(IBM_EHIP, "poisson_solve_static: no usable HIP device");
  void* sp = nullptr;
  if (scratch_address(dev, &sp) != IBM_OK)
    return ctx_fail(IBM_EHIP, "poisson_solve_static: hipGetSymbolAddress of the workspace failed");
  double* base = static_cast<double*>(sp);
  hipStream_t s = (hipStream_t)stream;
  const double dx = gr->lx / nx, dz = gr->lz / nz;
  for (int first = 0; first <= ny; first += FACES_CHUNK) {
    FaceChunk c;
    c.first = first;
    c.count = (ny + 1 - first < FACES_CHUNK) ? ny + 1 - first : FACES_CHUNK;
    for (int q = 0; q < c.count; ++q) c.v[q] = gr->y_faces[first + q];
    k_store_faces<<<1, 256, 0, s>>>(c, base + L.yf);
  }
  k_static_tables<<<1, 256, 0, s>>>(base, L, nx, ny, nz, dx, dz);
  GridView g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nxh = nx / 2 + 1;
  g.lx = gr->lx;
  g.lz = gr->lz;
  g.dx = dx;
  g.dz = dz;
  g.idx = 1.0 / dx;
  g.idz = 1.0 / dz;
  g.yf = base + L.yf;
  g.yc = base + L.yc;
  g.dy = base + L.dy;
  g.dyc = base + L.dyc;
  g.extuw = base + L.extuw;
  g.idy = base + L.idy;
  g.idyc = base + L.idyc;
  g.fw0 = base + L.fw0;
  g.fw1 = base + L.fw1;
  double sum_dy = 0.0;  // the context's sum, in its order
  for (int j = 0; j < ny; ++j) sum_dy += gr->y_faces[j + 1] - gr->y_faces[j];
  px.tw = reinterpret_cast<const double2*>(base + L.twx);
  pz.tw = reinterpret_cast<const double2*>(base + L.twz);
  PoissonArgs a{};
  a.px = &px;
  a.pz = &pz;
  a.lamx = base + L.lamx;
  a.lamz = base + L.lamz;
  a.ylo = base + L.ylo;
  a.yhi = base + L.yhi;
  a.spec = base + L.spec;
  a.sum_dy = sum_dy;
  a.vtot = dx * dz * (double)nx * (double)nz * sum_dy;
  a.flags = reinterpret_cast<uint32_t*>(base + L.flags);
  launch_poisson(nullptr, s, g, a, rhs, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 1.0,
                 phi);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return ctx_fail(IBM_EHIP, (std::string("poisson_solve_static: kernel launch: ") +
                               hipGetErrorString(e)).c_str());
  return IBM_OK;
}
