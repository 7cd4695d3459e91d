// Batched form: many independent simulations (each its own grid, state and
// body) advanced together on one GPU.  Small grids cannot fill the chip one
// at a time: each simulation's step is a chain of a few dozen small kernels
// whose cost is launch latency.  The batch gives every simulation its own
// HIP stream (forked from and joined back into the caller's stream), so the
// chains of different simulations run concurrently, and it can capture one
// whole batched step - every simulation's body transform and time step - into
// one HIP graph that is replayed each step with a single launch.  The body
// coefficients, which change every step, are read by the body kernels from a
// device buffer that is refreshed (one stream-ordered copy) before each step,
// so a replayed graph sees the new motion.
#include "ibm.h"

#include <cstring>
#include <vector>

#include "internal.h"

namespace ibm {
hipStream_t ctx_stream(ibm_ctx* c);
Prof* ctx_prof(ibm_ctx* c);
int ctx_prepare(ibm_ctx* c, const ibm_body* b, int32_t nb, double dt);
int ctx_fail(int code, const char* msg);
}  // namespace ibm

using namespace ibm;

struct ibm_batch {
  int n = 0;
  hipStream_t stream = nullptr;  // the caller's stream
  // the batch's own stream: the caller's stream may be one that cannot be
  // captured (the legacy default stream), so the batched work is forked from
  // it into this stream (ev_in) and joined back (ev_out)
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<ibm_ctx*> ctx;
  std::vector<hipStream_t> sstream;  // one per simulation (owned)
  std::vector<ibm_sim> sim;
  std::vector<ibm_body> body;
  double* coef_dev = nullptr;  // n x IBM_COEF_STRIDE
  static constexpr int NSTAGE = 4;
  double* coef_host[NSTAGE] = {};  // pinned staging of the coefficient upload
  hipEvent_t stage_ev[NSTAGE] = {};
  bool stage_used[NSTAGE] = {};
  int stage = 0;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> done;
  double prep_dt = -1.0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

#define BCHK(expr)                                                          \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return ctx_fail(IBM_EHIP, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
  } while (0)

static void drop_graph(ibm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static void free_batch(ibm_batch* b) {
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (hipStream_t s : b->sstream)
    if (s) (void)hipStreamSynchronize(s);
  if (b->own) (void)hipStreamSynchronize(b->own);
  drop_graph(b);
  for (ibm_ctx* c : b->ctx) ibm_destroy(c);
  if (b->own) (void)hipStreamDestroy(b->own);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  for (hipStream_t s : b->sstream)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->done)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (int k = 0; k < ibm_batch::NSTAGE; ++k) {
    if (b->coef_host[k]) (void)hipHostFree(b->coef_host[k]);
    if (b->stage_ev[k]) (void)hipEventDestroy(b->stage_ev[k]);
  }
  if (b->coef_dev) (void)hipFree(b->coef_dev);
  delete b;
}

// every simulation's body transform and step, forked from b->own and joined
// back into it; serial: each simulation waits for the previous one
static int enqueue(ibm_batch* b, double dt, bool serial) {
  BCHK(hipEventRecord(b->fork, b->own));
  for (int s = 0; s < b->n; ++s) {
    hipStream_t ss = b->sstream[s];
    BCHK(hipStreamWaitEvent(ss, (serial && s > 0) ? b->done[s - 1] : b->fork, 0));
    const ibm_sim& m = b->sim[s];
    launch_body_dev(ctx_prof(b->ctx[s]), ss, m.motion == IBM_MOTION_DEFORM, m.ref, m.nv,
                    b->coef_dev + (size_t)s * IBM_COEF_STRIDE, m.xyz, m.vel);
    ibm_state st = m.state;
    const int rc = ibm_step(b->ctx[s], &st, &b->body[s], 1, dt);
    if (rc) return rc;
    BCHK(hipEventRecord(b->done[s], ss));
  }
  if (serial) {
    BCHK(hipStreamWaitEvent(b->own, b->done[b->n - 1], 0));
  } else {
    for (int s = 0; s < b->n; ++s) BCHK(hipStreamWaitEvent(b->own, b->done[s], 0));
  }
  return IBM_OK;
}

extern "C" {

int ibm_batch_create(const ibm_grid* grids, const ibm_opts* opts, const ibm_sim* sims,
                     int32_t nsim, void* stream, ibm_batch** out) {
  if (!grids || !opts || !sims || !out || nsim < 1 || nsim > 4096)
    return ctx_fail(IBM_EINVAL, "ibm_batch_create: bad argument");
  *out = nullptr;
  for (int s = 0; s < nsim; ++s) {
    const ibm_sim& m = sims[s];
    if (!m.state.u || !m.state.v || !m.state.w || !m.state.p || m.nv < 0 || m.nt < 0 ||
        (m.nt > 0 && (!m.ref || !m.xyz || !m.vel || !m.tri)) ||
        (m.motion != IBM_MOTION_RIGID && m.motion != IBM_MOTION_DEFORM))
      return ctx_fail(IBM_EINVAL, "ibm_batch_create: bad simulation descriptor");
  }
  ibm_batch* b = new ibm_batch();
  b->n = nsim;
  b->stream = (hipStream_t)stream;
  b->sim.assign(sims, sims + nsim);
  b->ctx.assign(nsim, nullptr);
  b->sstream.assign(nsim, nullptr);
  b->done.assign(nsim, nullptr);
  int rc = IBM_OK;
#define BTRY(expr)                                                               \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      free_batch(b);                                                             \
      return ctx_fail(IBM_EHIP, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    }                                                                            \
  } while (0)
  for (int s = 0; s < nsim; ++s) {
    BTRY(hipStreamCreateWithFlags(&b->sstream[s], hipStreamNonBlocking));
    BTRY(hipEventCreateWithFlags(&b->done[s], hipEventDisableTiming));
    rc = ibm_create(&grids[s], &opts[s], b->sstream[s], &b->ctx[s]);
    if (rc) {
      b->ctx[s] = nullptr;
      free_batch(b);
      return rc;
    }
    ibm_body bd;
    bd.nv = sims[s].nv;
    bd.nt = sims[s].nt;
    bd.xyz = sims[s].xyz;
    bd.vel = sims[s].vel;
    bd.tri = sims[s].tri;
    b->body.push_back(bd);
  }
  BTRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  BTRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
  BTRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
  BTRY(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking));
  BTRY(hipMalloc(&b->coef_dev, sizeof(double) * IBM_COEF_STRIDE * (size_t)nsim));
  for (int k = 0; k < ibm_batch::NSTAGE; ++k) {
    BTRY(hipHostMalloc((void**)&b->coef_host[k], sizeof(double) * IBM_COEF_STRIDE * (size_t)nsim));
    BTRY(hipEventCreateWithFlags(&b->stage_ev[k], hipEventDisableTiming));
  }
#undef BTRY
  *out = b;
  return IBM_OK;
}

void ibm_batch_destroy(ibm_batch* b) {
  if (b) free_batch(b);
}

ibm_ctx* ibm_batch_context(ibm_batch* b, int32_t sim) {
  if (!b || sim < 0 || sim >= b->n) return nullptr;
  return b->ctx[sim];
}

int ibm_batch_step(ibm_batch* b, const double* coef, double dt, int32_t mode) {
  if (!b || !coef || !(dt > 0) || mode < IBM_BATCH_SERIAL || mode > IBM_BATCH_GRAPH)
    return ctx_fail(IBM_EINVAL, "ibm_batch_step: bad argument");
  if (dt != b->prep_dt) {
    // tables and body descriptors for this dt, outside any capture
    drop_graph(b);
    BCHK(hipStreamSynchronize(b->stream));
    BCHK(hipStreamSynchronize(b->own));
    for (int s = 0; s < b->n; ++s) {
      const int rc = ctx_prepare(b->ctx[s], &b->body[s], 1, dt);
      if (rc) return rc;
    }
    b->prep_dt = dt;
  }
  // coefficient upload through a pinned staging slot whose previous copy
  // has completed
  const int k = b->stage;
  b->stage = (k + 1) % ibm_batch::NSTAGE;
  if (b->stage_used[k]) BCHK(hipEventSynchronize(b->stage_ev[k]));
  const size_t bytes = sizeof(double) * IBM_COEF_STRIDE * (size_t)b->n;
  std::memcpy(b->coef_host[k], coef, bytes);
  BCHK(hipMemcpyAsync(b->coef_dev, b->coef_host[k], bytes, hipMemcpyHostToDevice, b->stream));
  BCHK(hipEventRecord(b->stage_ev[k], b->stream));
  b->stage_used[k] = true;
  BCHK(hipEventRecord(b->ev_in, b->stream));
  BCHK(hipStreamWaitEvent(b->own, b->ev_in, 0));
  if (mode != IBM_BATCH_GRAPH) {
    const int rc = enqueue(b, dt, mode == IBM_BATCH_SERIAL);
    if (rc) return rc;
  } else {
    if (!b->exec) {
      BCHK(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
      const int rc = enqueue(b, dt, false);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(b->own, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      BCHK(e);
      b->graph = g;
      BCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    BCHK(hipGraphLaunch(b->exec, b->own));
  }
  BCHK(hipEventRecord(b->ev_out, b->own));
  BCHK(hipStreamWaitEvent(b->stream, b->ev_out, 0));
  return IBM_OK;
}

int ibm_batch_check(ibm_batch* b, uint32_t* flags) {
  if (!b || !flags) return ctx_fail(IBM_EINVAL, "ibm_batch_check: bad argument");
  uint32_t all = 0;
  for (int s = 0; s < b->n; ++s) {
    uint32_t f = 0;
    const int rc = ibm_check(b->ctx[s], &f);
    if (rc) return rc;
    all |= f;
  }
  BCHK(hipStreamSynchronize(b->stream));
  *flags = all;
  return IBM_OK;
}

}  // extern "C"
