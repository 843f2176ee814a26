// Request loop over verified graph templates.
//
// CONTINUOUS mode: a worker thread admits queued requests in arrival order
// while their device buffers fit in the HBM budget and a slot is free, packs
// every admitted request into one device step (host-to-device copies, one
// batch launch over all their work items, device-to-host copies)
// on a stream with no step in flight, and retires steps as their completion
// events fire.  With n_streams >= 2, requests that arrive while a step runs
// start in a new step that overlaps it on the device.
//
// PLAIN mode: one request at a time, each with its own copies, its own
// kernel launch and a wait, the way a program calling process per frame
// would run them.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <set>
#include <thread>

#include "hvx_internal.h"
#include "kernels.h"

namespace hvx {

hvx_status prepare_graph(Graph* g);  // runtime.cpp

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device allocation.
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  bool init(size_t bytes) {
    if (hipMalloc((void**)&base, bytes) != hipSuccess) return false;
    size = bytes;
    free_[0] = bytes;
    return true;
  }
  void* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used += bytes;
      peak = std::max(peak, used);
      return base + off;
    }
    return nullptr;
  }
  void release(void* p, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    size_t off = (char*)p - base;
    used -= bytes;
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
  void destroy() {
    if (base) (void)hipFree(base);
    base = nullptr;
  }
};

struct Request {
  uint64_t tag;
  Graph* templ;
  const void* in;
  size_t in_pitch;
  void* out;
  size_t out_pitch;
  double t_submit;
  Value* vin;
  Value* vout;
  size_t in_row, out_row, in_bytes, out_bytes;  // device layout
  size_t d_in_pitch, d_out_pitch;
  void* d_in = nullptr;
  void* d_out = nullptr;
  bool fail = false;
};

struct StreamSlot {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  BatchImage* d_imgs = nullptr;
  uint16_t* d_items = nullptr;
  BatchImage* h_imgs = nullptr;  // pinned staging
  uint16_t* h_items = nullptr;
  size_t cap_imgs = 0, cap_items = 0;
  std::vector<Request*> reqs;
  bool busy = false;
};

struct Done {
  uint64_t tag;
  int32_t status;
  double latency;
};

struct Server : Object {
  int mode = 0;
  size_t budget = 0;
  uint32_t max_slots = 1;
  Arena arena;
  std::vector<StreamSlot> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::vector<Done> done;
  std::set<uint64_t> fail_tags;
  uint32_t in_flight = 0;
  uint32_t peak_in_flight = 0;
  int64_t submitted = 0, completed = 0, steps = 0;
  bool stop = false;
  std::thread worker;
};

static bool batchable(const Graph* g) {
  return g->plan && g->plan->groups.size() == 1 && is_strip_kind(g->plan->groups[0].kind);
}

static void finish(Server* sv, Request* r, int32_t status, double t) {
  if (r->d_in) sv->arena.release(r->d_in, r->in_bytes);
  if (r->d_out) sv->arena.release(r->d_out, r->out_bytes);
  sv->done.push_back({r->tag, status, t - r->t_submit});
  --sv->in_flight;
  ++sv->completed;
  delete r;
}

// Build the request's work description from its template with the request's
// device buffers bound in place of the template's images.
static void request_desc(Request* r, BatchImage* bi) {
  const Group& gr = r->templ->plan->groups[0];
  fill_fast_desc(r->templ, gr, bi);
  if (bi->kind == FK_EDGE) {
    bi->d.e.in = (const uint8_t*)r->d_in;
    bi->d.e.in_pitch = (int64_t)r->d_in_pitch;
    bi->d.e.out = (uint8_t*)r->d_out;
    bi->d.e.out_pitch = (int64_t)r->d_out_pitch;
    bi->d.e.phase = nullptr;
  } else if (bi->kind == FK_CORNER) {
    bi->d.c.in = (const uint8_t*)r->d_in;
    bi->d.c.in_pitch = (int64_t)r->d_in_pitch;
    bi->d.c.out = (uint8_t*)r->d_out;
    bi->d.c.out_pitch = (int64_t)r->d_out_pitch;
  } else if (bi->kind == FK_GAUSS5) {
    bi->d.g5.in = (const uint8_t*)r->d_in;
    bi->d.g5.in_pitch = (int64_t)r->d_in_pitch;
    bi->d.g5.out = (uint8_t*)r->d_out;
    bi->d.g5.out_pitch = (int64_t)r->d_out_pitch;
  }
}

static bool grow(StreamSlot& sl, size_t nimg, size_t nitems) {
  if (nimg > sl.cap_imgs) {
    if (sl.d_imgs) (void)hipFree(sl.d_imgs);
    if (sl.h_imgs) (void)hipHostFree(sl.h_imgs);
    sl.cap_imgs = std::max(nimg, 2 * sl.cap_imgs);
    if (hipMalloc((void**)&sl.d_imgs, sl.cap_imgs * sizeof(BatchImage)) != hipSuccess) return false;
    if (hipHostMalloc((void**)&sl.h_imgs, sl.cap_imgs * sizeof(BatchImage), 0) != hipSuccess) return false;
  }
  if (nitems > sl.cap_items) {
    if (sl.d_items) (void)hipFree(sl.d_items);
    if (sl.h_items) (void)hipHostFree(sl.h_items);
    sl.cap_items = std::max(nitems, 2 * sl.cap_items);
    if (hipMalloc((void**)&sl.d_items, sl.cap_items * sizeof(uint16_t)) != hipSuccess) return false;
    if (hipHostMalloc((void**)&sl.h_items, sl.cap_items * sizeof(uint16_t), 0) != hipSuccess) return false;
  }
  return true;
}

// Enqueue copies-in, the work, and copies-out of `reqs` on slot `sl`.
static bool launch_step(Server* sv, StreamSlot& sl, std::vector<Request*>& reqs) {
  hipStream_t s = sl.s;
  std::vector<Request*> live;
  for (Request* r : reqs)
    if (!r->fail) live.push_back(r);
  for (Request* r : live) {
    if (hipMemcpy2DAsync(r->d_in, r->d_in_pitch, r->in, r->in_pitch, r->in_row, r->vin->h, hipMemcpyHostToDevice,
                         s) != hipSuccess)
      return false;
  }
  if (sv->mode == HVX_SERVER_PLAIN) {
    for (Request* r : live) {
      if (batchable(r->templ)) {
        BatchImage bi;
        request_desc(r, &bi);
        const bool xcd = r->templ->plan->groups[0].xcd != 0;
        hipError_t e = bi.kind == FK_EDGE     ? launch_edge(bi.d.e, xcd, s)
                       : bi.kind == FK_CORNER ? launch_corner(bi.d.c, xcd, s)
                                              : launch_gauss5(bi.d.g5, xcd, s);
        if (e != hipSuccess) return false;
      }
    }
  } else if (!live.empty()) {
    size_t nitems = 0;
    std::vector<BatchImage> imgs(live.size());
    for (size_t i = 0; i < live.size(); ++i) {
      request_desc(live[i], &imgs[i]);
      nitems += imgs[i].nitems;
    }
    if (!grow(sl, imgs.size(), nitems)) return false;
    size_t first = 0;
    for (size_t i = 0; i < imgs.size(); ++i) {
      imgs[i].first_item = (int)first;
      for (int k = 0; k < imgs[i].nitems; ++k) sl.h_items[first + k] = (uint16_t)i;
      first += imgs[i].nitems;
    }
    memcpy(sl.h_imgs, imgs.data(), imgs.size() * sizeof(BatchImage));
    if (hipMemcpyAsync(sl.d_imgs, sl.h_imgs, imgs.size() * sizeof(BatchImage), hipMemcpyHostToDevice, s) != hipSuccess)
      return false;
    if (hipMemcpyAsync(sl.d_items, sl.h_items, nitems * sizeof(uint16_t), hipMemcpyHostToDevice, s) != hipSuccess)
      return false;
    int kinds = 0;
    for (const BatchImage& bi : imgs) kinds |= kind_bit(bi);
    // one wave per work item (the direct form measured faster than the
    // persistent one on every batch shape served here)
    if (launch_batch(sl.d_imgs, sl.d_items, (int)nitems, nullptr, 1, false, kinds, s) != hipSuccess)
      return false;
  }
  for (Request* r : live) {
    if (hipMemcpy2DAsync(r->out, r->out_pitch, r->d_out, r->d_out_pitch, r->out_row, r->vout->h,
                         hipMemcpyDeviceToHost, s) != hipSuccess)
      return false;
  }
  if (hipEventRecord(sl.done, s) != hipSuccess) return false;
  sl.reqs = reqs;
  sl.busy = true;
  ++sv->steps;
  return true;
}

static void worker_main(Server* sv) {
  (void)hipSetDevice(sv->ctx->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (true) {
    bool progress = false;
    // retire finished steps
    for (StreamSlot& sl : sv->slots) {
      if (!sl.busy) continue;
      hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      const double t = now_s();
      for (Request* r : sl.reqs) finish(sv, r, r->fail ? HVX_ERROR_DEVICE : (q == hipSuccess ? 0 : HVX_ERROR_DEVICE), t);
      sl.reqs.clear();
      sl.busy = false;
      progress = true;
    }
    if (sv->stop && sv->queue.empty() && sv->in_flight == 0) break;
    // admit in arrival order while memory and slots allow
    std::vector<Request*> admitted;
    const bool plain = sv->mode == HVX_SERVER_PLAIN;
    StreamSlot* free_slot = nullptr;
    for (StreamSlot& sl : sv->slots)
      if (!sl.busy) {
        free_slot = &sl;
        break;
      }
    while (free_slot && !sv->queue.empty() && sv->in_flight < sv->max_slots) {
      Request* r = sv->queue.front();
      if (r->fail) {
        sv->queue.pop_front();
        ++sv->in_flight;
        admitted.push_back(r);
        if (plain) break;
        continue;
      }
      void* a = sv->arena.alloc(r->in_bytes);
      void* b = a ? sv->arena.alloc(r->out_bytes) : nullptr;
      if (!a || !b) {
        if (a) sv->arena.release(a, r->in_bytes);
        break;  // head of line waits for memory
      }
      r->d_in = a;
      r->d_out = b;
      sv->queue.pop_front();
      ++sv->in_flight;
      sv->peak_in_flight = std::max(sv->peak_in_flight, sv->in_flight);
      admitted.push_back(r);
      if (plain) break;
    }
    if (!admitted.empty()) {
      if (!launch_step(sv, *free_slot, admitted)) {
        const double t = now_s();
        (void)hipStreamSynchronize(free_slot->s);
        for (Request* r : admitted) finish(sv, r, HVX_ERROR_DEVICE, t);
        free_slot->busy = false;
        free_slot->reqs.clear();
      }
      progress = true;
      if (plain) {
        // plain execution waits for each request before taking the next
        lk.unlock();
        (void)hipStreamSynchronize(free_slot->s);
        lk.lock();
        continue;
      }
    }
    if (!progress) sv->cv.wait_for(lk, std::chrono::microseconds(50));
  }
}

void destroy_server_object(Object* o) {
  Server* sv = (Server*)o;
  {
    std::lock_guard<std::mutex> l(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (Request* r : sv->queue) delete r;
  for (StreamSlot& sl : sv->slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.s) (void)hipStreamDestroy(sl.s);
    if (sl.d_imgs) (void)hipFree(sl.d_imgs);
    if (sl.d_items) (void)hipFree(sl.d_items);
    if (sl.h_imgs) (void)hipHostFree(sl.h_imgs);
    if (sl.h_items) (void)hipHostFree(sl.h_items);
  }
  sv->arena.destroy();
  registry_remove(sv);
  delete sv;
}

}  // namespace hvx

using namespace hvx;

extern "C" {

hvx_status hvx_server_create(hvx_context ctx, int mode, size_t budget, uint32_t max_slots, uint32_t n_streams,
                             hvx_server* out) {
  if (!registry_check(ctx, T_CONTEXT)) return HVX_ERROR_INVALID_REFERENCE;
  Context* c = (Context*)ctx;
  if (!out) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null output handle");
  *out = nullptr;
  if (mode != HVX_SERVER_CONTINUOUS && mode != HVX_SERVER_PLAIN)
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "unknown server mode %d", mode);
  if (max_slots == 0 || n_streams == 0 || n_streams > 16)
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "need max_slots >= 1 and 1 <= n_streams <= 16");
  if (budget == 0) return set_error(c, HVX_ERROR_NO_MEMORY, "HBM budget is zero");
  hvx_status s = ensure_device(c);
  if (s) return s;
  Server* sv = new Server();
  sv->type = T_SERVER;
  sv->ctx = c;
  sv->mode = mode;
  sv->budget = budget;
  sv->max_slots = max_slots;
  if (!sv->arena.init(budget)) {
    delete sv;
    return set_error(c, HVX_ERROR_NO_MEMORY, "cannot reserve %zu bytes of device memory", budget);
  }
  sv->slots.resize(mode == HVX_SERVER_PLAIN ? 1 : n_streams);
  for (StreamSlot& sl : sv->slots) {
    // default priority streams only
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      registry_add(sv);
      destroy_server_object(sv);
      return set_error(c, HVX_ERROR_DEVICE, "server stream setup failed");
    }
  }
  registry_add(sv);
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    c->children.push_back(sv);
  }
  sv->worker = std::thread(worker_main, sv);
  *out = (hvx_server)sv;
  return HVX_SUCCESS;
}

hvx_status hvx_server_submit(hvx_server hs, hvx_graph templ, const void* in, size_t in_pitch, void* out,
                             size_t out_pitch, uint64_t tag) {
  if (!registry_check(hs, T_SERVER)) return HVX_ERROR_INVALID_REFERENCE;
  Server* sv = (Server*)hs;
  if (!registry_check(templ, T_GRAPH)) return set_error(sv->ctx, HVX_ERROR_INVALID_REFERENCE, "invalid template");
  Graph* g = (Graph*)templ;
  if (!g->verified) {
    hvx_status s = verify_graph(g);
    if (s) return s;
  }
  if (!batchable(g))
    return set_error(sv->ctx, HVX_ERROR_NOT_SUPPORTED, "template must be a single fused kernel of a served kind");
  if (g->plan->groups[0].inputs.size() != 1 || g->plan->groups[0].outputs.size() != 1)
    return set_error(sv->ctx, HVX_ERROR_NOT_SUPPORTED, "template must have one input and one output image");
  if (!in || !out) return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "null host buffer");
  const Group& gr = g->plan->groups[0];
  Request* r = new Request();
  r->tag = tag;
  r->templ = g;
  r->in = in;
  r->in_pitch = in_pitch;
  r->out = out;
  r->out_pitch = out_pitch;
  r->vin = &g->plan->vals[gr.v_in];
  r->vout = &g->plan->vals[gr.v_out];
  r->in_row = (size_t)r->vin->w * df_bytes(r->vin->df);
  r->out_row = (size_t)r->vout->w * df_bytes(r->vout->df);
  if (in_pitch < r->in_row || out_pitch < r->out_row) {
    delete r;
    return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "host pitch smaller than a row");
  }
  r->d_in_pitch = (r->in_row + 63) / 64 * 64;
  r->d_out_pitch = (r->out_row + 63) / 64 * 64;
  r->in_bytes = r->d_in_pitch * r->vin->h;
  r->out_bytes = r->d_out_pitch * r->vout->h;
  if (r->in_bytes + r->out_bytes + 512 > sv->budget) {
    delete r;
    return set_error(sv->ctx, HVX_ERROR_NO_MEMORY, "request needs more than the whole HBM budget");
  }
  {
    std::lock_guard<std::mutex> l(sv->mu);
    r->fail = sv->fail_tags.count(tag) > 0;
    r->t_submit = now_s();
    sv->queue.push_back(r);
    ++sv->submitted;
  }
  sv->cv.notify_all();
  return HVX_SUCCESS;
}

hvx_status hvx_server_poll(hvx_server hs, uint64_t* tags, int32_t* statuses, double* latency, uint32_t max,
                           uint32_t* n) {
  if (!registry_check(hs, T_SERVER)) return HVX_ERROR_INVALID_REFERENCE;
  Server* sv = (Server*)hs;
  if (!n || (max && (!tags || !statuses || !latency)))
    return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "null output");
  std::lock_guard<std::mutex> l(sv->mu);
  uint32_t k = 0;
  while (k < max && k < sv->done.size()) {
    tags[k] = sv->done[k].tag;
    statuses[k] = sv->done[k].status;
    latency[k] = sv->done[k].latency;
    ++k;
  }
  sv->done.erase(sv->done.begin(), sv->done.begin() + k);
  *n = k;
  return HVX_SUCCESS;
}

hvx_status hvx_server_drain(hvx_server hs) {
  if (!registry_check(hs, T_SERVER)) return HVX_ERROR_INVALID_REFERENCE;
  Server* sv = (Server*)hs;
  while (true) {
    {
      std::lock_guard<std::mutex> l(sv->mu);
      if (sv->queue.empty() && sv->in_flight == 0) return HVX_SUCCESS;
    }
    sv->cv.notify_all();
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
}

hvx_status hvx_server_stats(hvx_server hs, int what, int64_t* out) {
  if (!registry_check(hs, T_SERVER)) return HVX_ERROR_INVALID_REFERENCE;
  Server* sv = (Server*)hs;
  if (!out) return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "null output");
  std::lock_guard<std::mutex> l(sv->mu);
  switch (what) {
    case 0: *out = sv->submitted; break;
    case 1: *out = sv->completed; break;
    case 2: *out = (int64_t)sv->arena.peak; break;
    case 3: *out = sv->peak_in_flight; break;
    case 4: *out = sv->steps; break;
    case 5: *out = (int64_t)sv->arena.used; break;
    default: return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown statistic %d", what);
  }
  return HVX_SUCCESS;
}

hvx_status hvx_server_inject_failure(hvx_server hs, uint64_t tag) {
  if (!registry_check(hs, T_SERVER)) return HVX_ERROR_INVALID_REFERENCE;
  Server* sv = (Server*)hs;
  std::lock_guard<std::mutex> l(sv->mu);
  sv->fail_tags.insert(tag);
  return HVX_SUCCESS;
}

hvx_status hvx_release_server(hvx_server* ps) {
  if (!ps || !registry_check(*ps, T_SERVER)) return HVX_ERROR_INVALID_REFERENCE;
  Server* sv = (Server*)*ps;
  Context* c = sv->ctx;
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    auto& v = c->children;
    v.erase(std::remove(v.begin(), v.end(), (Object*)sv), v.end());
  }
  destroy_server_object(sv);
  *ps = nullptr;
  return HVX_SUCCESS;
}

}  // extern "C"
