// gdg_server.cpp -- the request server of include/gdg.h: continuous batching
// of independent simulations on one GPU.
//
// Memory: the caller's pool holds, at its start, the device work list and the
// status copies; the rest is handed out first-fit (256-byte granules) to the
// workspaces of admitted requests and returned when they finish.  Each
// resident request is an ordinary context (gdg_create on its pool range, the
// server's stream), so every per-request rule -- CFL time step, capped last
// step, restart after a violation, admissibility checks -- is the one of the
// single-mesh path.  What the server adds is the batched launch: one captured
// graph of several device-driven steps whose persistent kernels walk the row
// blocks of all resident requests.
//
// Streams: the batched graph runs on the caller's stream; admissions (set-up,
// state upload) and the host-driven redo of a halted step run on a second
// stream of the same priority, so that a request is admitted while a launch
// is in flight; the next launch waits for that stream through an event.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "gdg.h"
#include "gdg_internal.h"

using namespace gdg;

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Streams on which the graphs of solo requests run side by side: a large
// request alone at the per-step floor of its dependent launches leaves most
// of the chip idle, so up to this many of them overlap.
constexpr int kSoloStreams = 3;

// First-fit allocator over [0, size) in 256-byte granules; free ranges are
// kept by offset and merged with their neighbours on release.
class PoolAlloc {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto &f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Req {
  uint64_t ticket = 0;
  gdg_mesh_desc mesh{};
  gdg_params prm{};
  std::vector<double> U;  // initial state until admission, final state after
  std::vector<double> vx; // general cells: the request's vertices (mesh.vertices points here)
  std::vector<int8_t> bcc; // boundary parts: their kinds (mesh.bc_cells points here)
  double t_final = 0.0;
  size_t bytes = 0, off = 0;
  gdg_ctx *ctx = nullptr;
  bool solo = false;  // runs its own single-mesh graph instead of the batched kernels
  int state = GDG_REQ_PENDING;
  int status = GDG_OK;
  double t = 0.0;
  int64_t steps = 0, restarts = 0, ndofs = 0;
  double submit_s = 0.0, admit_s = 0.0, done_s = 0.0;
};

size_t list_bytes() { return align256(sizeof(BatchList)); }
size_t status_bytes() { return align256(sizeof(Ctl) * kMaxBatch); }

}  // namespace

struct gdg_server {
  gdg_server_desc d{};
  char *pool = nullptr;
  size_t pool_bytes = 0;
  hipStream_t stream = nullptr;      // batched launches
  hipStream_t adm_stream = nullptr;  // admissions, restarts, retirements (the requests' contexts)
  hipStream_t cap_stream = nullptr;
  hipStream_t solo_stream[kSoloStreams] = {};  // solo requests' graphs, side by side
  hipEvent_t solo_ev[kSoloStreams] = {};       // joins each solo stream into the status copy
  hipEvent_t done_ev = nullptr;      // after the status copy of the launch in flight
  hipEvent_t adm_ev = nullptr;       // joins the admission stream into the next launch
  hipGraphExec_t gexec = nullptr;
  BatchList *dlist = nullptr;  // device work list (pool start)
  Ctl *dstat = nullptr;        // device status copies
  Ctl *hstat = nullptr;        // pinned host mirror of the status copies
  BatchList *hlist = nullptr;  // host image of the work list
  PoolAlloc alloc;
  size_t base = 0;             // first pool byte for workspaces
  int grid = 0;
  std::deque<Req *> pending;
  std::vector<Req *> resident;  // admitted, in work-list order
  std::vector<Req *> staged;    // admitted while a launch was in flight: join the next work list
  std::vector<Req *> launched;  // the work list of the launch in flight
  bool list_dirty = true;
  bool in_flight = false;
  std::unordered_map<uint64_t, Req *> reqs;
  uint64_t next_ticket = 1;
  std::chrono::steady_clock::time_point t0;
  std::string err;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

gdg_status fail_hip(gdg_server *s, const char *what, hipError_t e) {
  s->err = std::string(what) + ": " + hipGetErrorString(e);
  return GDG_E_DEVICE;
}

#define SRVCHK(s, call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return fail_hip((s), #call, e_); \
  } while (0)

void release(gdg_server *s, Req *q) {
  if (q->ctx) {
    gdg_destroy(q->ctx);
    q->ctx = nullptr;
    s->alloc.release(q->off - s->base, q->bytes);
  }
}

void fail_req(gdg_server *s, Req *q, gdg_status st, const std::string &why) {
  q->state = GDG_REQ_FAILED;
  q->status = st;
  q->done_s = s->now();
  if (!why.empty()) s->err = "request " + std::to_string(q->ticket) + ": " + why;
  release(s, q);
  std::vector<double>().swap(q->U);
}

void take_stats(Req *q) { ctx_counts(q->ctx, &q->t, &q->steps, &q->restarts); }

// Copies the final state to the request's host buffer and frees its range.
gdg_status finish_req(gdg_server *s, Req *q) {
  q->U.assign((size_t)(q->mesh.dim + 2) * (size_t)q->ndofs, 0.0);
  const gdg_status st = gdg_download_state(q->ctx, q->U.data(), 0);
  if (st != GDG_OK) {
    fail_req(s, q, st, ctx_error(q->ctx));
    return GDG_OK;
  }
  q->state = GDG_REQ_DONE;
  q->done_s = s->now();
  release(s, q);
  return GDG_OK;
}

// Steps 1-3 of a pump, once the launch in flight has completed: take every
// request's control block, redo halted steps, retire finished requests.
gdg_status process(gdg_server *s) {
  if (!s->in_flight) return GDG_OK;
  s->in_flight = false;
  for (size_t r = 0; r < s->launched.size(); ++r) {
    Req *q = s->launched[r];
    const Ctl c = s->hstat[r];
    if (c.bad_flag) {
      const gdg_status st = flag_status(q->ctx, c.bad_flag, "a stage output left the admissible set");
      fail_req(s, q, st, ctx_error(q->ctx));
      continue;
    }
    ctx_sync(q->ctx, c);
    if (c.cfl_flag) {
      const gdg_status st = ctx_restart(q->ctx, c, q->t_final);
      if (st != GDG_OK) {
        fail_req(s, q, st, ctx_error(q->ctx));
        continue;
      }
    }
    take_stats(q);
    if (!(q->t < q->t_final))
      if (gdg_status st = finish_req(s, q)) return st;
  }
  std::vector<Req *> keep;
  for (Req *q : s->resident)
    if (q->state == GDG_REQ_RUNNING) keep.push_back(q);
  if (keep.size() != s->resident.size()) s->list_dirty = true;
  s->resident.swap(keep);
  return GDG_OK;
}

// Step 4: admission in arrival order while a slot and pool room are free, on
// the admission stream (the batched launch may still be running).
void admit(gdg_server *s) {
  while (!s->pending.empty() && (int)(s->resident.size() + s->staged.size()) < s->d.max_slots) {
    Req *q = s->pending.front();
    size_t off = 0;
    if (!s->alloc.alloc(q->bytes, &off)) break;  // the head waits for room
    s->pending.pop_front();
    q->off = s->base + off;
    q->admit_s = s->now();
    gdg_status st = gdg_create(&q->mesh, &q->prm, s->pool + q->off, q->bytes, s->adm_stream, &q->ctx);
    if (st != GDG_OK) {
      q->ctx = nullptr;
      s->alloc.release(off, q->bytes);
      fail_req(s, q, st, gdg_last_error(nullptr));
      continue;
    }
    st = gdg_upload_state(q->ctx, q->U.data(), 0);
    if (st != GDG_OK) {
      fail_req(s, q, st, ctx_error(q->ctx));
      continue;
    }
    std::vector<double>().swap(q->U);
    q->state = GDG_REQ_RUNNING;
    q->solo = s->d.solo_dofs > 0 && q->ndofs >= s->d.solo_dofs;
    if (!(0.0 < q->t_final)) {
      take_stats(q);
      finish_req(s, q);
      continue;
    }
    if (ctx_arm(q->ctx, q->t_final) != 0) {
      fail_req(s, q, GDG_E_DEVICE, "kernel launch failed: set run");
      continue;
    }
    s->staged.push_back(q);
  }
}

// Staged admissions join the work list of the next launch.
void merge_staged(gdg_server *s) {
  if (s->staged.empty()) return;
  for (Req *q : s->staged) s->resident.push_back(q);
  s->staged.clear();
  s->list_dirty = true;
}

gdg_status ensure_graph(gdg_server *s) {
  if (s->gexec) return GDG_OK;
  if (!s->cap_stream) SRVCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  SRVCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = launch_batch_steps(s->d.dim, s->d.degree, s->d.precision == GDG_MIXED ? 1 : 0, s->dlist, s->dstat,
                                    s->d.steps_per_graph, s->grid, s->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
  if (rc != 0 || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    s->err = std::string("graph capture failed: ") + hipGetErrorString(e);
    return GDG_E_DEVICE;
  }
  e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    s->gexec = nullptr;
    return fail_hip(s, "graph instantiation", e);
  }
  return GDG_OK;
}

// Device resources of the server, set up at the first launch (creation and
// submission touch no device).
gdg_status ensure_device(gdg_server *s) {
  if (s->hstat) return GDG_OK;
  int dev = 0, cus = 0;
  SRVCHK(s, hipGetDevice(&dev));
  SRVCHK(s, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  // a plain stream: the default priority, as the caller's
  SRVCHK(s, hipStreamCreateWithFlags(&s->adm_stream, hipStreamNonBlocking));
  SRVCHK(s, hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming));
  SRVCHK(s, hipEventCreateWithFlags(&s->adm_ev, hipEventDisableTiming));
  for (int k = 0; k < kSoloStreams; ++k) {
    SRVCHK(s, hipStreamCreateWithFlags(&s->solo_stream[k], hipStreamNonBlocking));
    SRVCHK(s, hipEventCreateWithFlags(&s->solo_ev[k], hipEventDisableTiming));
  }
  SRVCHK(s, hipHostMalloc((void **)&s->hstat, sizeof(Ctl) * kMaxBatch, hipHostMallocDefault));
  // one-wavefront workgroups: eight per CU keep every SIMD busy with two
  // waves while leaving room for the register budget of the sweeps
  s->grid = (cus > 0 ? cus : 256) * 8;
  return GDG_OK;
}

// Step 5: refresh the device work list if the batched set changed, launch
// the batched graph and then each solo request's own graph after the
// admission stream's work, and queue the status copy (batched requests
// first, then the solo ones, in `launched` order).  Called only when no
// launch is in flight, so the caller's stream is idle.
gdg_status launch(gdg_server *s) {
  if (s->resident.empty()) return GDG_OK;
  if (gdg_status st = ensure_device(s)) return st;
  std::vector<Req *> batch, solo;
  for (Req *q : s->resident) (q->solo ? solo : batch).push_back(q);
  const int nb = (int)batch.size();
  if (s->list_dirty) {
    BatchList &L = *s->hlist;
    L.nreq = nb;
    L.tile_begin[0] = 0;
    for (int r = 0; r < nb; ++r) {
      BatchEntry &E = L.e[r];
      E.A = ctx_kargs(batch[r]->ctx);
      ctx_stage_bufs(batch[r]->ctx, E.sb);
      L.tile_begin[r + 1] = L.tile_begin[r] + E.A.nblocks;
    }
    L.ntiles = L.tile_begin[nb];
    const size_t bytes = offsetof(BatchList, e) + sizeof(BatchEntry) * (size_t)nb;
    SRVCHK(s, hipMemcpyAsync(s->dlist, s->hlist, bytes, hipMemcpyHostToDevice, s->stream));
    SRVCHK(s, hipStreamSynchronize(s->stream));  // the host image may change before the next launch
    s->list_dirty = false;
  }
  if (nb > 0)
    if (gdg_status st = ensure_graph(s)) return st;
  SRVCHK(s, hipEventRecord(s->adm_ev, s->adm_stream));
  SRVCHK(s, hipStreamWaitEvent(s->stream, s->adm_ev, 0));
  if (nb > 0) SRVCHK(s, hipGraphLaunch(s->gexec, s->stream));
  // solo request r runs on solo stream r % kSoloStreams after the admission
  // stream's work; the status copy waits for every solo stream used
  const int nstreams = solo.size() < (size_t)kSoloStreams ? (int)solo.size() : kSoloStreams;
  for (int k = 0; k < nstreams; ++k) SRVCHK(s, hipStreamWaitEvent(s->solo_stream[k], s->adm_ev, 0));
  for (size_t r = 0; r < solo.size(); ++r) {
    hipStream_t st = s->solo_stream[r % kSoloStreams];
    if (ctx_launch_steps(solo[r]->ctx, st) != 0) {
      s->err = std::string("solo request launch failed: ") + ctx_error(solo[r]->ctx);
      return GDG_E_DEVICE;
    }
    SRVCHK(s, hipMemcpyAsync(s->dstat + nb + r, ctx_dev_ctl(solo[r]->ctx), sizeof(Ctl), hipMemcpyDeviceToDevice, st));
  }
  for (int k = 0; k < nstreams; ++k) {
    SRVCHK(s, hipEventRecord(s->solo_ev[k], s->solo_stream[k]));
    SRVCHK(s, hipStreamWaitEvent(s->stream, s->solo_ev[k], 0));
  }
  const size_t n = batch.size() + solo.size();
  SRVCHK(s, hipMemcpyAsync(s->hstat, s->dstat, sizeof(Ctl) * n, hipMemcpyDeviceToHost, s->stream));
  SRVCHK(s, hipEventRecord(s->done_ev, s->stream));
  s->launched = batch;
  s->launched.insert(s->launched.end(), solo.begin(), solo.end());
  s->in_flight = true;
  return GDG_OK;
}

// Whether the launch in flight (if any) has completed, without waiting.
gdg_status flight_done(gdg_server *s, bool *done) {
  *done = true;
  if (!s->in_flight) return GDG_OK;
  const hipError_t e = hipEventQuery(s->done_ev);
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();  // not an error: clear it for later calls
    *done = false;
    return GDG_OK;
  }
  if (e != hipSuccess) return fail_hip(s, "hipEventQuery", e);
  return GDG_OK;
}

bool desc_ok(const gdg_server_desc *d) {
  return d && d->dim >= 1 && d->dim <= 3 && d->degree >= 1 && d->degree <= 3 && !(d->degree == 3 && d->dim == 3) &&
         (d->precision == GDG_FP64 || d->precision == GDG_MIXED) && d->max_slots >= 1 &&
         d->max_slots <= kMaxBatch && d->steps_per_graph >= 1 && d->steps_per_graph <= 64 && d->solo_dofs >= 0;
}

}  // namespace

extern "C" {

gdg_status gdg_server_overhead_bytes(const gdg_server_desc *desc, size_t *bytes) {
  if (!desc_ok(desc) || !bytes) return GDG_E_INVALID;
  *bytes = list_bytes() + status_bytes();
  return GDG_OK;
}

gdg_status gdg_server_create(const gdg_server_desc *desc, void *dev_pool, size_t pool_bytes, void *hip_stream,
                             gdg_server **out) {
  if (!out) return GDG_E_INVALID;
  *out = nullptr;
  if (!desc_ok(desc) || !dev_pool || ((uintptr_t)dev_pool & 255)) return GDG_E_INVALID;
  const size_t over = list_bytes() + status_bytes();
  if (pool_bytes <= over) return GDG_E_NOMEM;
  gdg_server *s = new gdg_server();
  s->d = *desc;
  s->pool = (char *)dev_pool;
  s->pool_bytes = pool_bytes;
  s->stream = (hipStream_t)hip_stream;
  s->dlist = (BatchList *)s->pool;
  s->dstat = (Ctl *)(s->pool + list_bytes());
  s->base = over;
  s->alloc.reset(pool_bytes - over);
  s->hlist = new BatchList();
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return GDG_OK;
}

gdg_status gdg_server_submit(gdg_server *s, const gdg_mesh_desc *mesh, const gdg_params *prm, const double *U0,
                             double t_final, uint64_t *ticket) {
  if (!s || !mesh || !prm || !U0 || !ticket) return GDG_E_INVALID;
  if (mesh->ucells > 0 || mesh->continuous) {
    s->err = "unstructured meshes and continuous elements are not served";
    return GDG_E_INVALID;
  }
  if (prm->integrator != GDG_SSPRK3) {
    s->err = "the server steps with SSP-RK3 only";
    return GDG_E_INVALID;
  }
  if (mesh->data_kind == GDG_DATA_STEP_START) {
    s->err = "step-start boundary data are not served";
    return GDG_E_INVALID;
  }
  if (mesh->dim != s->d.dim || mesh->degree != s->d.degree || prm->precision != s->d.precision) {
    s->err = "request outside the server's class (dim, degree, precision)";
    return GDG_E_INVALID;
  }
  size_t bytes = 0;
  if (gdg_workspace_bytes(mesh, prm, &bytes) != GDG_OK) {
    s->err = "invalid mesh description or scheme constants";
    return GDG_E_INVALID;
  }
  if (align256(bytes) > s->pool_bytes - s->base) {
    s->err = "request workspace exceeds the memory pool";
    return GDG_E_BUDGET;
  }
  Req *q = new Req();
  q->ticket = s->next_ticket++;
  q->mesh = *mesh;
  if (mesh->vertices) {
    size_t npts = 1;
    const int g = mesh->map_degree == 2 ? 2 : 1;
    for (int e = 0; e < mesh->dim; ++e) npts *= (size_t)(g * mesh->cells[e] + 1);
    q->vx.assign(mesh->vertices, mesh->vertices + npts * mesh->dim);
    q->mesh.vertices = q->vx.data();
  }
  if (mesh->bc_cells) {
    // one entry per cell face of each non-periodic box face (gdg.h)
    int64_t n = 0;
    for (int f = 0; f < 2 * mesh->dim; ++f) {
      if (mesh->bc[f] == GDG_BC_PERIODIC) continue;
      int64_t cnt = 1;
      for (int g = 0; g < mesh->dim; ++g)
        if (g != f / 2) cnt *= mesh->cells[g];
      n += cnt;
    }
    q->bcc.assign(mesh->bc_cells, mesh->bc_cells + n);
    q->mesh.bc_cells = q->bcc.data();
  }
  q->prm = *prm;
  q->t_final = t_final;
  q->bytes = bytes;
  int64_t ncells = 1;
  for (int e = 0; e < mesh->dim; ++e) ncells *= mesh->cells[e];
  int nloc = 1;
  for (int e = 0; e < mesh->dim; ++e) nloc *= mesh->degree + 1;
  q->ndofs = ncells * nloc;
  q->U.assign(U0, U0 + (size_t)(mesh->dim + 2) * (size_t)q->ndofs);
  q->submit_s = s->now();
  s->pending.push_back(q);
  s->reqs[q->ticket] = q;
  *ticket = q->ticket;
  return GDG_OK;
}

gdg_status gdg_server_sync(gdg_server *s) {
  if (!s) return GDG_E_INVALID;
  if (s->in_flight) SRVCHK(s, hipEventSynchronize(s->done_ev));
  return process(s);
}

gdg_status gdg_server_pump(gdg_server *s, int32_t *resident, int32_t *pending) {
  if (!s) return GDG_E_INVALID;
  if (gdg_status st = ensure_device(s)) return st;
  bool done = true;
  if (gdg_status st = flight_done(s, &done)) return st;
  if (done) {
    if (gdg_status st = process(s)) return st;
    admit(s);
    merge_staged(s);
    if (gdg_status st = launch(s)) return st;
  } else {
    admit(s);  // overlaps the launch in flight; joins the next one
  }
  if (resident) *resident = (int32_t)(s->resident.size() + s->staged.size());
  if (pending) *pending = (int32_t)s->pending.size();
  return GDG_OK;
}

gdg_status gdg_server_poll(const gdg_server *s, uint64_t ticket, gdg_request_info *info) {
  if (!s || !info) return GDG_E_INVALID;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return GDG_E_INVALID;
  const Req *q = it->second;
  info->state = q->state;
  info->status = q->status;
  info->t = q->t;
  info->steps = q->steps;
  info->restarts = q->restarts;
  info->ndofs = q->ndofs;
  info->submit_s = q->submit_s;
  info->admit_s = q->admit_s;
  info->done_s = q->done_s;
  return GDG_OK;
}

gdg_status gdg_server_result(gdg_server *s, uint64_t ticket, double *U) {
  if (!s || !U) return GDG_E_INVALID;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->state != GDG_REQ_DONE) return GDG_E_INVALID;
  Req *q = it->second;
  std::memcpy(U, q->U.data(), q->U.size() * sizeof(double));
  s->reqs.erase(it);
  delete q;
  return GDG_OK;
}

void gdg_server_destroy(gdg_server *s) {
  if (!s) return;
  if (s->hstat || !s->resident.empty()) (void)hipStreamSynchronize(s->stream);
  if (s->adm_stream) (void)hipStreamSynchronize(s->adm_stream);
  for (int k = 0; k < kSoloStreams; ++k)
    if (s->solo_stream[k]) (void)hipStreamSynchronize(s->solo_stream[k]);
  for (auto &kv : s->reqs) {
    if (kv.second->ctx) gdg_destroy(kv.second->ctx);
    delete kv.second;
  }
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->done_ev) (void)hipEventDestroy(s->done_ev);
  if (s->adm_ev) (void)hipEventDestroy(s->adm_ev);
  if (s->adm_stream) (void)hipStreamDestroy(s->adm_stream);
  for (int k = 0; k < kSoloStreams; ++k) {
    if (s->solo_ev[k]) (void)hipEventDestroy(s->solo_ev[k]);
    if (s->solo_stream[k]) (void)hipStreamDestroy(s->solo_stream[k]);
  }
  if (s->hstat) (void)hipHostFree(s->hstat);
  delete s->hlist;
  delete s;
}

const char *gdg_server_last_error(const gdg_server *s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
