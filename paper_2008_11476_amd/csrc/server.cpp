// Request loop over verified graph templates.
//
// A request runs a template on images of its own: host frames (copied into
// device buffers the server takes from its HBM budget, and back), or frames
// already in device memory (run in place).  A template whose plan is one
// strip kernel (edge, with or without Phase; corner; Gaussian5x5) joins the
// batch launch of a step; any other template runs its own plan on the
// request's images, its intermediates in a scratch block taken from the
// budget.
//
// CONTINUOUS mode: a worker thread admits queued requests in arrival order
// while their device memory fits in the HBM budget and a slot is free, packs
// every admitted request into one device step (host-to-device copies, one
// batch launch over all their work items plus the plans of the other
// templates, device-to-host copies) on a stream with no step in flight, and
// retires steps as their completion events fire.  With n_streams >= 2,
// requests that arrive while a step runs start in a new step that overlaps
// it on the device.
//
// PLAIN mode: one request at a time, each with its own copies, its own
// kernel launches and a wait, the way a program calling process per frame
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

// One non-virtual image of a request's template, bound to the request's memory.
struct Binding {
  int v = -1;                // plan value of the template image
  bool input = false;        // a graph input (copied in for host requests)
  const void* host = nullptr;  // host requests: the caller's pixels
  size_t host_pitch = 0;
  void* dev = nullptr;       // device memory the request runs on
  size_t dev_pitch = 0;
  size_t row = 0, h = 0;     // bytes per row, rows
  size_t bytes = 0;          // arena bytes (host requests)
};

struct Request {
  uint64_t tag;
  Graph* templ;
  double t_submit;
  bool device = false;  // frames already in device memory: no copies, nothing from the arena
  std::vector<Binding> io;
  char* scratch = nullptr;  // intermediates of a non-batched template
  size_t scratch_bytes = 0;
  Bind bind;
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

static void release_memory(Server* sv, Request* r) {
  if (!r->device)
    for (Binding& b : r->io)
      if (b.dev) {
        sv->arena.release(b.dev, b.bytes);
        b.dev = nullptr;
      }
  if (r->scratch) sv->arena.release(r->scratch, r->scratch_bytes);
  r->scratch = nullptr;
}

// Device memory of a request from the arena (host buffers, the scratch
// block); false, with nothing kept, when it does not fit now.
static bool take_memory(Server* sv, Request* r) {
  bool ok = true;
  if (!r->device)
    for (Binding& b : r->io) {
      b.dev = sv->arena.alloc(b.bytes);
      if (!b.dev) {
        ok = false;
        break;
      }
    }
  if (ok && r->scratch_bytes) {
    r->scratch = (char*)sv->arena.alloc(r->scratch_bytes);
    ok = r->scratch != nullptr;
  }
  if (!ok) {
    release_memory(sv, r);
    return false;
  }
  r->bind.ptr.assign(r->templ->plan->vals.size(), nullptr);
  r->bind.pitch.assign(r->templ->plan->vals.size(), 0);
  for (const Binding& b : r->io) {
    r->bind.ptr[b.v] = b.dev;
    r->bind.pitch[b.v] = (int64_t)b.dev_pitch;
  }
  r->bind.scratch = r->scratch;
  return true;
}

static void finish(Server* sv, Request* r, int32_t status, double t) {
  release_memory(sv, r);
  sv->done.push_back({r->tag, status, t - r->t_submit});
  --sv->in_flight;
  ++sv->completed;
  delete r;
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
  for (Request* r : live)
    if (!r->device)
      for (const Binding& b : r->io)
        if (b.input && hipMemcpy2DAsync(b.dev, b.dev_pitch, b.host, b.host_pitch, b.row, b.h, hipMemcpyHostToDevice,
                                        s) != hipSuccess)
          return false;
  std::vector<BatchImage> imgs;
  for (Request* r : live) {
    if (batchable(r->templ) && sv->mode == HVX_SERVER_CONTINUOUS) {
      imgs.emplace_back();
      fill_fast_desc(r->templ, r->templ->plan->groups[0], &imgs.back(), 0, &r->bind);
    } else if (schedule_bound(r->templ, s, &r->bind) != HVX_SUCCESS) {
      return false;
    }
  }
  if (!imgs.empty()) {
    size_t nitems = 0;
    for (const BatchImage& bi : imgs) nitems += bi.nitems;
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
  for (Request* r : live)
    if (!r->device)
      for (const Binding& b : r->io)
        if (!b.input && hipMemcpy2DAsync((void*)b.host, b.host_pitch, b.dev, b.dev_pitch, b.row, b.h,
                                         hipMemcpyDeviceToHost, s) != hipSuccess)
          return false;
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
      if (!take_memory(sv, r)) break;  // head of line waits for memory
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

// Checks a request against its template and queues it.  `bind` gives, for
// each non-virtual image of the template, the request's memory (host or
// device) and its pitch.
static hvx_status submit_request(Server* sv, Graph* g, const std::vector<std::pair<Image*, std::pair<void*, size_t>>>& bind,
                                 bool device, uint64_t tag) {
  if (!g->verified) {
    hvx_status s = verify_graph(g);
    if (s) return s;
  }
  hvx_status st = prepare_graph(g);
  if (st) return st;
  const Plan& p = *g->plan;
  auto* r = new Request();
  r->tag = tag;
  r->templ = g;
  r->device = device;
  std::vector<int> seen(p.vals.size(), 0);
  for (size_t v = 0; v < p.vals.size(); ++v) {
    const Value& val = p.vals[v];
    if (val.is_virtual || !val.live) continue;
    if (val.df == DF_BUF) {
      delete r;
      return set_error(sv->ctx, HVX_ERROR_NOT_SUPPORTED, "templates with global operator results are not served");
    }
    Binding b;
    b.v = (int)v;
    b.input = val.producer < 0;
    b.row = (size_t)val.w * df_bytes(val.df);
    b.h = val.h;
    bool found = false;
    for (const auto& x : bind)
      if (x.first == val.img) {
        if (found) {
          delete r;
          return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "an image is bound twice");
        }
        found = true;
        if (!x.second.first || x.second.second < b.row) {
          delete r;
          return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "null buffer or pitch smaller than a row");
        }
        if (device) {
          if (x.second.second % 64 || ((uintptr_t)x.second.first & 15)) {
            delete r;
            return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS,
                             "device buffers need a 16-byte aligned base and a pitch that is a multiple of 64");
          }
          b.dev = x.second.first;
          b.dev_pitch = x.second.second;
        } else {
          b.host = x.second.first;
          b.host_pitch = x.second.second;
          b.dev_pitch = (b.row + 63) / 64 * 64;
          b.bytes = b.dev_pitch * b.h;
        }
      }
    if (!found) {
      delete r;
      return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "an image of the template is not bound");
    }
    r->io.push_back(b);
  }
  size_t need = 0;
  for (const Binding& b : r->io) need += (b.bytes + 255) & ~(size_t)255;
  if (!batchable(g)) r->scratch_bytes = g->scratch_total;
  need += (r->scratch_bytes + 255) & ~(size_t)255;
  if (need > sv->budget) {
    delete r;
    return set_error(sv->ctx, HVX_ERROR_NO_MEMORY, "request needs more than the whole HBM budget");
  }
  // the server's device pointers are set at admission
  if (!device)
    for (Binding& b : r->io) b.dev = nullptr;
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
  if (!in || !out) return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "null host buffer");
  // the template's one input and one output image
  Image *iim = nullptr, *oim = nullptr;
  int nin = 0, nout = 0;
  for (const Value& val : g->plan->vals) {
    if (val.is_virtual || !val.live) continue;
    if (val.producer < 0) {
      iim = val.img;
      ++nin;
    } else {
      oim = val.img;
      ++nout;
    }
  }
  if (nin != 1 || nout != 1)
    return set_error(sv->ctx, HVX_ERROR_NOT_SUPPORTED,
                     "this call serves templates with one input and one output image (see hvx_server_submit_bound)");
  return submit_request(sv, g, {{iim, {(void*)in, in_pitch}}, {oim, {out, out_pitch}}}, false, tag);
}

hvx_status hvx_server_submit_bound(hvx_server hs, hvx_graph templ, const hvx_binding* bindings, uint32_t n,
                                   int memory, uint64_t tag) {
  if (!registry_check(hs, T_SERVER)) return HVX_ERROR_INVALID_REFERENCE;
  Server* sv = (Server*)hs;
  if (!registry_check(templ, T_GRAPH)) return set_error(sv->ctx, HVX_ERROR_INVALID_REFERENCE, "invalid template");
  if (memory != HVX_MEMORY_HOST && memory != HVX_MEMORY_DEVICE)
    return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown memory kind %d", memory);
  if (n && !bindings) return set_error(sv->ctx, HVX_ERROR_INVALID_PARAMETERS, "null bindings");
  std::vector<std::pair<Image*, std::pair<void*, size_t>>> bind;
  for (uint32_t i = 0; i < n; ++i) {
    if (!registry_check(bindings[i].image, T_IMAGE))
      return set_error(sv->ctx, HVX_ERROR_INVALID_REFERENCE, "binding %u: invalid image", i);
    bind.push_back({(Image*)bindings[i].image, {bindings[i].ptr, bindings[i].pitch}});
  }
  return submit_request(sv, (Graph*)templ, bind, memory == HVX_MEMORY_DEVICE, tag);
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
