// Device runtime: launching verified graphs, batches, autotuning, tune cache.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <map>
#include <set>
#include <sstream>

#include "global.h"
#include "codegen.h"
#include "hvx_internal.h"
#include "kernels.h"

namespace hvx {

int32_t edge_threshold_not(double t);  // verify.cpp

hvx_status ensure_device(Context* ctx) {
  std::lock_guard<std::recursive_mutex> l(ctx->mu);
  if (ctx->dev_ready) {
    (void)hipSetDevice(ctx->device);
    return HVX_SUCCESS;
  }
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) return set_error(ctx, HVX_ERROR_DEVICE, "no HIP device available");
  if (ctx->device >= n) return set_error(ctx, HVX_ERROR_DEVICE, "device %d out of range (%d devices)", ctx->device, n);
  e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return set_error(ctx, HVX_ERROR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
    ctx->num_cus = prop.multiProcessorCount;
    ctx->dev_name = prop.gcnArchName;
  }
  ctx->dev_ready = true;
  return HVX_SUCCESS;
}

void free_graph_device(Graph* g) {
  if (g->scheduled && g->last_stream != (void*)-1) (void)hipStreamSynchronize((hipStream_t)g->last_stream);
  if (g->scratch_base) (void)hipFree(g->scratch_base);
  if (g->dev_progs) (void)hipFree(g->dev_progs);
  g->dev_progs = nullptr;
  g->scratch_base = nullptr;
  g->scratch_total = 0;
  g->scratch_off.clear();
  g->scratch_pitch.clear();
  g->ws_off.clear();
  g->prepared = false;
  g->scheduled = false;
}

// Device copies of the generic programs and one scratch block holding every
// materialised value (rows pitched to 64 bytes, each value 256-byte aligned).
static hvx_status ensure_scratch(Graph* g) {
  Plan& p = *g->plan;
  if (g->prepared) return HVX_SUCCESS;
  for (const Group& gr : p.groups)
    if (gr.gen) {
      const hipError_t e = gen_load(gr.gen, g->ctx->device);
      if (e != hipSuccess)
        return set_error(g->ctx, HVX_ERROR_DEVICE, "cannot load a generated kernel: %s", hipGetErrorString(e));
    }
  std::vector<GProg> progs(p.groups.size());
  for (size_t i = 0; i < p.groups.size(); ++i) progs[i] = p.groups[i].prog;
  if (hipMalloc((void**)&g->dev_progs, progs.size() * sizeof(GProg)) != hipSuccess ||
      hipMemcpy(g->dev_progs, progs.data(), progs.size() * sizeof(GProg), hipMemcpyHostToDevice) != hipSuccess) {
    if (g->dev_progs) (void)hipFree(g->dev_progs);
    g->dev_progs = nullptr;
    return set_error(g->ctx, HVX_ERROR_NO_MEMORY, "cannot upload kernel programs");
  }
  g->scratch_off.assign(p.vals.size(), 0);
  g->scratch_pitch.assign(p.vals.size(), 0);
  size_t total = 0;
  for (size_t v = 0; v < p.vals.size(); ++v) {
    if (!p.vals[v].materialize) continue;
    const size_t pitch = ((size_t)p.vals[v].w * df_bytes(p.vals[v].df) + 63) / 64 * 64;
    g->scratch_off[v] = total;
    g->scratch_pitch[v] = pitch;
    total += (pitch * p.vals[v].h + 255) & ~(size_t)255;
  }
  // workspace of the generated kernels that reduce: one slot of partial
  // results per work-group (tile)
  g->ws_off.assign(p.groups.size(), 0);
  for (size_t gi = 0; gi < p.groups.size(); ++gi) {
    const Group& gr = p.groups[gi];
    if (!gr.gen || gen_batchable(gr.gen)) continue;
    g->ws_off[gi] = total;
    const size_t bytes = (size_t)gen_blocks(gr.gen, gr.prog.w, gr.prog.h) * red_slot_words(gr.prog) * 4;
    total += (bytes + 255) & ~(size_t)255;
  }
  if (total && hipMalloc((void**)&g->scratch_base, total) != hipSuccess) {
    g->scratch_base = nullptr;
    free_graph_device(g);
    return set_error(g->ctx, HVX_ERROR_NO_MEMORY, "cannot allocate %zu bytes for intermediate images", total);
  }
  g->scratch_total = total;
  g->prepared = true;
  return HVX_SUCCESS;
}

// Device address and pitch of value v: a non-virtual image's own memory (or
// the request's, under a binding), a materialised intermediate in the
// scratch block (the graph's, or the binding's).
static void value_ptr(const Graph* g, int v, void** ptr, int64_t* pitch, const Bind* b = nullptr) {
  const Value& val = g->plan->vals[v];
  if (!val.is_virtual) {
    if (b && v < (int)b->ptr.size() && b->ptr[v]) {
      *ptr = b->ptr[v];
      *pitch = b->pitch[v];
    } else {
      *ptr = val.img->ptr;
      *pitch = (int64_t)val.img->pitch;
    }
  } else if (v < (int)g->scratch_pitch.size() && g->scratch_pitch[v]) {
    char* base = b && b->scratch ? b->scratch : g->scratch_base;
    *ptr = base + g->scratch_off[v];
    *pitch = (int64_t)g->scratch_pitch[v];
  } else {
    *ptr = nullptr;
    *pitch = 0;
  }
}

static const LOp* find_op(const Plan& p, const Group& gr, int kind) {
  for (int o : gr.ops)
    if (p.ops[o].kind == kind) return &p.ops[o];
  return nullptr;
}

static std::string tune_key(const Graph* g) { return g->ctx->dev_name + "|" + graph_signature(g); }

int default_rows(const Group& gr, int num_cus) {
  // enough work items to give every CU several waves, without letting the
  // halo rows (footprint on each side) dominate a work item
  const int sp = gr.kind == FK_CORNER ? 62 * 4 : kStripPx;
  const int nstrips = ((int)gr.w + sp - 1) / sp;
  int64_t target = 4LL * num_cus;
  int64_t rows = ((int64_t)gr.h * nstrips) / std::max<int64_t>(1, target);
  int r = 4;
  while (r * 2 <= rows && r < 64) r *= 2;
  return r;
}

int rows_for(const Graph* g, const Group& gr) {
  if (gr.rows > 0) return gr.rows;
  auto it = g->ctx->tune.find(tune_key(g));
  if (it != g->ctx->tune.end() && it->second.rows > 0) return it->second.rows;
  return default_rows(gr, g->ctx->num_cus);
}

static int xcd_for(const Graph* g, const Group& gr) {
  if (gr.rows > 0) return gr.xcd;
  auto it = g->ctx->tune.find(tune_key(g));
  if (it != g->ctx->tune.end() && it->second.rows > 0) return it->second.xcd;
  return gr.xcd;
}

static int strip_px(int kind) { return kind == FK_CORNER ? 62 * 4 : kStripPx; }

static StripGrid strip_grid(const Group& gr, int rows) {
  StripGrid s;
  s.w = (int)gr.w;
  s.h = (int)gr.h;
  s.rows = std::max(1, rows);
  s.nstrips = (s.w + strip_px(gr.kind) - 1) / strip_px(gr.kind);
  s.nbands = (s.h + s.rows - 1) / s.rows;
  return s;
}

int64_t fast_items(const Group& gr) { return (int64_t)gr.prog.tiles_x; }

void fill_fast_desc(const Graph* g, const Group& gr, BatchImage* bi, int rows_override, const Bind* b) {
  const Plan& p = *g->plan;
  memset(bi, 0, sizeof *bi);
  bi->kind = gr.kind;
  const int rows = rows_override > 0 ? rows_override : rows_for(g, gr);
  void* ptr;
  int64_t pitch;
  if (gr.kind == FK_EDGE) {
    EdgeDesc& d = bi->d.e;
    d.g = strip_grid(gr, rows);
    value_ptr(g, gr.v_in, &ptr, &pitch, b);
    d.in = (const uint8_t*)ptr;
    d.in_pitch = pitch;
    value_ptr(g, gr.v_out, &ptr, &pitch, b);
    d.out = (uint8_t*)ptr;
    d.out_pitch = pitch;
    if (gr.v_aux >= 0) {
      value_ptr(g, gr.v_aux, &ptr, &pitch, b);
      d.phase = (uint8_t*)ptr;
      d.phase_pitch = pitch;
    }
    const LOp* ga = find_op(p, gr, OP_GAUSS3);
    const LOp* sx = find_op(p, gr, OP_SOBEL_X);
    const LOp* th = find_op(p, gr, OP_THRESHOLD);
    d.b0 = ga->border;
    d.c0 = (int)std::min<uint32_t>(ga->bconst, 255);
    d.b1 = sx->border;
    d.c1 = (int)std::min<uint32_t>(sx->bconst, 255);
    d.thr_not = edge_threshold_not(th->dval);
    d.tv4 = 0x01010101u * (uint32_t)(th->tv & 0xFF);
    d.fv4 = 0x01010101u * (uint32_t)(th->fv & 0xFF);
    bi->nitems = d.g.nstrips * d.g.nbands;
  } else if (gr.kind == FK_CORNER) {
    CornerDesc& d = bi->d.c;
    d.g = strip_grid(gr, rows);
    value_ptr(g, gr.v_in, &ptr, &pitch, b);
    d.in = (const uint8_t*)ptr;
    d.in_pitch = pitch;
    value_ptr(g, gr.v_out, &ptr, &pitch, b);
    d.out = (uint8_t*)ptr;
    d.out_pitch = pitch;
    const LOp* sx = find_op(p, gr, OP_SOBEL_X);
    const LOp* bx = find_op(p, gr, OP_BOX5F);
    const LOp* hr = find_op(p, gr, OP_HARRIS);
    const LOp* th = find_op(p, gr, OP_THRESHOLD);
    d.b0 = sx->border;
    d.c0 = (int)std::min<uint32_t>(sx->bconst, 255);
    d.b1 = bx->border;
    d.c1 = (float)bx->bconst;
    d.k = hr->k;
    float f = (float)th->dval;
    if ((double)f > th->dval) f = nextafterf(f, -INFINITY);
    d.thr = f;
    d.tv4 = 0x01010101u * (uint32_t)(th->tv & 0xFF);
    d.fv4 = 0x01010101u * (uint32_t)(th->fv & 0xFF);
    bi->nitems = d.g.nstrips * d.g.nbands;
  } else if (gr.kind == FK_GAUSS5) {
    Gauss5Desc& d = bi->d.g5;
    d.g = strip_grid(gr, rows);
    value_ptr(g, gr.v_in, &ptr, &pitch, b);
    d.in = (const uint8_t*)ptr;
    d.in_pitch = pitch;
    d.uyvy = p.vals[gr.v_in].df == DF_UYVY;
    value_ptr(g, gr.v_out, &ptr, &pitch, b);
    d.out = (uint8_t*)ptr;
    d.out_pitch = pitch;
    const LOp* g5 = find_op(p, gr, OP_GAUSS5);
    d.b0 = g5->border;
    d.c0 = (int)std::min<uint32_t>(g5->bconst, 255);
    bi->nitems = d.g.nstrips * d.g.nbands;
  }
}

// One global operator over an image in memory (group kind FK_GLOBAL), with
// the streaming kernels of the immediate-mode calls.
static hipError_t launch_global_group(Graph* g, const Group& gr, hipStream_t s, const Bind* b) {
  const Plan& p = *g->plan;
  const LOp& o = p.ops[gr.ops[0]];
  void* ptr;
  int64_t pitch;
  value_ptr(g, o.in[0], &ptr, &pitch, b);
  const Value& iv = p.vals[o.in[0]];
  GlobalImg im{(const uint8_t*)ptr, pitch, (int32_t)iv.w, (int32_t)iv.h, df_bytes(iv.df)};
  void* out;
  int64_t unused;
  value_ptr(g, o.out, &out, &unused, b);
  switch (o.kind) {
    case OP_HISTOGRAM: return launch_histogram(im, (int)o.gp[0], (int)o.gp[1], (int)o.gp[2], (uint32_t*)out, s);
    case OP_MINMAX: return launch_min_max(im, (int32_t*)out, s);
    case OP_MMCOUNT: {
      hipError_t e = launch_min_max_count(im, (int32_t*)out, s);
      return e != hipSuccess ? e : launch_zero_words((int32_t*)out + 4, 2, s);  // no locations stored (yet)
    }
    case OP_SUMS: return launch_mean_std_dev(im, out, s);
    case OP_EQHIST: return launch_equalize_mapping(im, out, s);
    case OP_MMLOCS: {
      void* mm;
      value_ptr(g, o.in[1], &mm, &unused, b);
      const uint32_t cap = o.gp[0];
      hipError_t e = launch_extreme_locs(im, (int32_t*)mm, (uint32_t*)out, (uint32_t*)out + 2 * cap, cap, s);
      return e != hipSuccess ? e : launch_clamp_slots((int32_t*)mm, cap, s);
    }
  }
  return hipErrorInvalidValue;
}

// The device pointers and pitches a generic group's kernel reads and writes.
static hvx_status fill_io(Graph* g, const Group& gr, IOTable* io, const Bind* b) {
  memset(io, 0, sizeof *io);
  for (int i = 0; i < gr.prog.nvals; ++i) {
    const GVal& v = gr.prog.vals[i];
    if (v.io < 0) continue;
    value_ptr(g, gr.gvals[i], &io->ptr[v.io], &io->pitch[v.io], b);
    if (!io->ptr[v.io]) return set_error(g->ctx, HVX_ERROR_DEVICE, "unbound image in plan");
  }
  return HVX_SUCCESS;
}

static hvx_status launch_group(Graph* g, const Group& gr, hipStream_t s, const Bind* b) {
  hipError_t e = hipSuccess;
  const int gi = (int)(&gr - g->plan->groups.data());
  if (gr.kind == FK_GENERIC) {
    IOTable io;
    hvx_status fs = fill_io(g, gr, &io, b);
    if (fs) return fs;
    // global operators reduced by the kernel: starting values before it,
    // final values after it, in the same stream
    const GProg& P = gr.prog;
    for (int i = 0; i < P.nops && e == hipSuccess; ++i)
      if (is_reduce_op(P.ops[i].kind))
        e = launch_reduce_init(P.ops[i].kind, io.ptr[P.vals[P.ops[i].out].io], P.ops[i].p0, s);
    if (e == hipSuccess && gr.gen && !gen_batchable(gr.gen)) {
      // a generated kernel that reduces leaves one slot of partial results
      // per work-group; a second kernel merges them into the results
      char* base = b && b->scratch ? b->scratch : g->scratch_base;
      uint32_t* ws = (uint32_t*)(base + g->ws_off[gi]);
      e = gen_launch(gr.gen, g->ctx->device, P, g->dev_progs + gi, io, g->ctx->num_cus, s, ws);
      if (e == hipSuccess)
        e = launch_merge_partials(g->dev_progs + gi, io, ws, (int)gen_blocks(gr.gen, P.w, P.h), red_slot_words(P), s);
    } else if (e == hipSuccess) {
      e = gr.gen ? gen_launch(gr.gen, g->ctx->device, P, g->dev_progs + gi, io, g->ctx->num_cus, s, nullptr)
                 : launch_generic(P, g->dev_progs + gi, io, g->ctx->num_cus, s);
    }
    for (int i = 0; i < P.nops && e == hipSuccess; ++i)
      if (is_reduce_op(P.ops[i].kind)) {
        void* out = io.ptr[P.vals[P.ops[i].out].io];
        e = launch_reduce_finish(P.ops[i].kind, out, (long long)P.w * P.h, s);
        if (e == hipSuccess && P.ops[i].kind == OP_MMCOUNT) e = launch_zero_words((int32_t*)out + 4, 2, s);
      }
  } else if (gr.kind == FK_GLOBAL) {
    e = launch_global_group(g, gr, s, b);
  } else {
    BatchImage bi;
    fill_fast_desc(g, gr, &bi, 0, b);
    const bool xcd = xcd_for(g, gr) != 0;
    if (gr.kind == FK_EDGE) e = launch_edge(bi.d.e, xcd, s);
    else if (gr.kind == FK_CORNER) e = launch_corner(bi.d.c, xcd, s);
    else if (gr.kind == FK_GAUSS5) e = launch_gauss5(bi.d.g5, xcd, s);
    else return set_error(g->ctx, HVX_ERROR_NOT_SUPPORTED, "no kernel for group kind %d", gr.kind);
  }
  if (e != hipSuccess) return set_error(g->ctx, HVX_ERROR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
  return HVX_SUCCESS;
}

hvx_status prepare_graph(Graph* g) {
  hvx_status s = ensure_device(g->ctx);
  if (s) return s;
  return ensure_scratch(g);
}

hvx_status schedule_bound(Graph* g, void* stream, const Bind* b) {
  hvx_status s = prepare_graph(g);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  for (const Group& gr : g->plan->groups) {
    s = launch_group(g, gr, st, b);
    if (s) return s;
  }
  // The graph waits for its own schedules (hvx_graph_wait, release).  A
  // bound run belongs to its caller (the server), which waits for its own
  // streams and may destroy them before the graph: the graph must not keep
  // such a stream.
  if (!b) {
    g->last_stream = stream;
    g->scheduled = true;
  }
  return HVX_SUCCESS;
}

hvx_status schedule_graph(Graph* g, void* stream) { return schedule_bound(g, stream, nullptr); }

// ---- batches --------------------------------------------------------------------

struct Batch : Object {
  std::vector<Graph*> graphs;
  std::vector<Graph*> separate;  // graphs not expressible as batch work items
  std::vector<BatchImage> imgs;
  std::vector<uint16_t> item_img;
  BatchImage* d_imgs = nullptr;
  uint16_t* d_item_img = nullptr;
  unsigned* d_counter = nullptr;
  int total = 0, grid = 0;
  bool persistent = true, use_graph = true;
  hipGraph_t hg = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t alg_bytes = 0;
  int rows_override = 0;  // rows per work item for every image (0: each graph's own)
  int kinds = 0;          // bit set of the kinds in the single batch launch
  // chains of generated kernels shared by several graphs: one launch per kernel
  struct GenSet {
    const GenKernel* k = nullptr;
    std::vector<GenBatchImage> imgs;
    GenBatchImage* d = nullptr;
    long long blocks = 0;
  };
  std::vector<GenSet> gensets;
  void* last_stream = nullptr;
  bool scheduled = false;
};

static void batch_free_device(Batch* b) {
  if (b->scheduled) (void)hipStreamSynchronize((hipStream_t)b->last_stream);
  b->scheduled = false;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->hg) (void)hipGraphDestroy(b->hg);
  b->exec = nullptr;
  b->hg = nullptr;
  if (b->d_imgs) (void)hipFree(b->d_imgs);
  if (b->d_item_img) (void)hipFree(b->d_item_img);
  for (auto& gs : b->gensets)
    if (gs.d) (void)hipFree(gs.d);
  b->gensets.clear();
  if (b->d_counter) (void)hipFree(b->d_counter);
  b->d_imgs = nullptr;
  b->d_item_img = nullptr;
  b->d_counter = nullptr;
}

void destroy_batch_object(Object* o) {
  Batch* b = (Batch*)o;
  batch_free_device(b);
  registry_remove(b);
  delete b;
}

static double kind_cost(const BatchImage& bi) {
  switch (bi.kind) {
    case FK_EDGE: return bi.d.e.phase ? 3.0 * bi.d.e.g.rows : 2.0 * bi.d.e.g.rows;
    case FK_CORNER: return 4.0 * bi.d.c.g.rows;
    case FK_GAUSS5: return 1.0 * bi.d.g5.g.rows;
  }
  return 1.0;
}

static hvx_status batch_build(Batch* b) {
  Context* c = b->ctx;
  batch_free_device(b);
  b->imgs.clear();
  b->separate.clear();
  b->alg_bytes = 0;
  for (Graph* g : b->graphs) {
    if (!g->verified) {
      hvx_status s = verify_graph(g);
      if (s) return s;
    }
    hvx_status s = prepare_graph(g);
    if (s) return s;
    b->alg_bytes += g->plan->alg_bytes;
    const auto& gs = g->plan->groups;
    if (gs.size() == 1 && is_strip_kind(gs[0].kind)) {
      BatchImage bi;
      fill_fast_desc(g, gs[0], &bi, b->rows_override);
      b->imgs.push_back(bi);
    } else {
      b->separate.push_back(g);
    }
  }
  // graphs whose plan is a chain of generated kernels: the graphs with the
  // same chain run it as one launch per kernel over all their tiles (a work
  // list of image and tile), the chain's kernels in plan order, so every
  // group still runs after the groups it reads
  {
    auto chain_of = [](const Graph* g) {
      std::vector<const GenKernel*> ks;
      for (const Group& gr : g->plan->groups) {
        if (gr.kind != FK_GENERIC || !gr.gen || !gen_batchable(gr.gen)) return std::vector<const GenKernel*>();
        ks.push_back(gr.gen);
      }
      return ks;
    };
    std::map<std::vector<const GenKernel*>, std::vector<Graph*>> by_chain;
    for (Graph* g : b->separate) {
      const auto ks = chain_of(g);
      if (!ks.empty()) by_chain[ks].push_back(g);
    }
    std::vector<Graph*> rest;
    for (Graph* g : b->separate) {
      const auto ks = chain_of(g);
      if (ks.empty() || by_chain[ks].size() < 2) rest.push_back(g);
    }
    for (auto& kv : by_chain) {
      if (kv.second.size() < 2) continue;
      for (size_t stage = 0; stage < kv.first.size(); ++stage) {
        Batch::GenSet set;
        set.k = kv.first[stage];
        for (Graph* g : kv.second) {
          const Group& gr = g->plan->groups[stage];
          GenBatchImage im;
          memset(&im, 0, sizeof im);
          hvx_status st = fill_io(g, gr, &im.io, nullptr);
          if (st) return st;
          im.w = gr.prog.w;
          im.h = gr.prog.h;
          im.block0 = (int32_t)set.blocks;
          set.blocks += gen_blocks(set.k, gr.prog.w, gr.prog.h);
          if (set.blocks > 0x7FFFFFFF) return set_error(c, HVX_ERROR_NOT_SUPPORTED, "batch launch too large");
          set.imgs.push_back(im);
        }
        b->gensets.push_back(std::move(set));
      }
    }
    b->separate.swap(rest);
    for (auto& set : b->gensets) {
      const size_t bytes = set.imgs.size() * sizeof(GenBatchImage);
      if (hipMalloc((void**)&set.d, bytes) != hipSuccess) return set_error(c, HVX_ERROR_NO_MEMORY, "batch tables");
      if (hipMemcpy(set.d, set.imgs.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
        return set_error(c, HVX_ERROR_DEVICE, "batch table upload");
    }
  }
  // heaviest items first, so the last items handed out are the cheapest
  std::stable_sort(b->imgs.begin(), b->imgs.end(),
                   [](const BatchImage& x, const BatchImage& y) { return kind_cost(x) > kind_cost(y); });
  if (b->imgs.size() > 65535) return set_error(c, HVX_ERROR_NOT_SUPPORTED, "at most 65535 images per batch");
  b->item_img.clear();
  int first = 0;
  for (size_t i = 0; i < b->imgs.size(); ++i) {
    b->imgs[i].first_item = first;
    for (int k = 0; k < b->imgs[i].nitems; ++k) b->item_img.push_back((uint16_t)i);
    first += b->imgs[i].nitems;
  }
  b->total = first;
  b->kinds = 0;
  for (const BatchImage& bi : b->imgs) b->kinds |= kind_bit(bi);
  b->grid = std::max(1, std::min(b->total, c->num_cus * batch_waves_per_cu(b->kinds)));
  if (!b->imgs.empty()) {
    if (hipMalloc((void**)&b->d_imgs, b->imgs.size() * sizeof(BatchImage)) != hipSuccess ||
        hipMalloc((void**)&b->d_item_img, b->item_img.size() * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc((void**)&b->d_counter, batch_counter_bytes()) != hipSuccess) {
      batch_free_device(b);
      return set_error(c, HVX_ERROR_NO_MEMORY, "batch descriptors");
    }
    hipError_t e = hipMemcpy(b->d_imgs, b->imgs.data(), b->imgs.size() * sizeof(BatchImage), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(b->d_item_img, b->item_img.data(), b->item_img.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->d_counter, 0, batch_counter_bytes());
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      batch_free_device(b);
      return set_error(c, HVX_ERROR_DEVICE, "batch upload: %s", hipGetErrorString(e));
    }
  }
  return HVX_SUCCESS;
}

// kernel launches of one schedule: the single batch launch plus the plans of
// the graphs it cannot hold
static int64_t batch_launches(const Batch* b) {
  int64_t k = b->total > 0 ? 1 : 0;
  k += (int64_t)b->gensets.size();
  for (Graph* g : b->separate) k += (int64_t)g->plan->groups.size();
  return k;
}

static hvx_status batch_enqueue(Batch* b, hipStream_t s) {
  if (b->total > 0) {
    hipError_t e = launch_batch(b->d_imgs, b->d_item_img, b->total, b->d_counter, b->grid, b->persistent, b->kinds, s);
    if (e != hipSuccess) return set_error(b->ctx, HVX_ERROR_DEVICE, "batch launch: %s", hipGetErrorString(e));
  }
  for (const auto& set : b->gensets) {
    hipError_t e = gen_launch_batch(set.k, b->ctx->device, set.d, (int)set.imgs.size(), set.blocks, s);
    if (e != hipSuccess) return set_error(b->ctx, HVX_ERROR_DEVICE, "generated batch launch: %s", hipGetErrorString(e));
  }
  for (Graph* g : b->separate) {
    hvx_status st = HVX_SUCCESS;
    for (const Group& gr : g->plan->groups) {
      st = launch_group(g, gr, s, nullptr);
      if (st) return st;
    }
  }
  return HVX_SUCCESS;
}

}  // namespace hvx

using namespace hvx;

extern "C" {

hvx_status hvx_batch_create(hvx_context ctx, const hvx_graph* graphs, uint32_t n, hvx_batch* out) {
  if (!registry_check(ctx, T_CONTEXT)) return HVX_ERROR_INVALID_REFERENCE;
  Context* c = (Context*)ctx;
  if (!out || (!graphs && n)) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null argument");
  *out = nullptr;
  for (uint32_t i = 0; i < n; ++i)
    if (!registry_check(graphs[i], T_GRAPH) || ((Graph*)graphs[i])->ctx != c)
      return set_error(c, HVX_ERROR_INVALID_REFERENCE, "batch graph %u is invalid", i);
  hvx_status s = ensure_device(c);
  if (s) return s;
  Batch* b = new Batch();
  b->type = T_BATCH;
  b->ctx = c;
  for (uint32_t i = 0; i < n; ++i) b->graphs.push_back((Graph*)graphs[i]);
  s = batch_build(b);
  if (s) {
    batch_free_device(b);
    delete b;
    return s;
  }
  registry_add(b);
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    c->children.push_back(b);
  }
  *out = (hvx_batch)b;
  return HVX_SUCCESS;
}

hvx_status hvx_batch_refresh(hvx_batch hb) {
  if (!registry_check(hb, T_BATCH)) return HVX_ERROR_INVALID_REFERENCE;
  return batch_build((Batch*)hb);
}

hvx_status hvx_batch_schedule(hvx_batch hb, void* stream) {
  if (!registry_check(hb, T_BATCH)) return HVX_ERROR_INVALID_REFERENCE;
  Batch* b = (Batch*)hb;
  hipStream_t s = (hipStream_t)stream;
  hvx_status st = ensure_device(b->ctx);
  if (st) return st;
  const int64_t launches = batch_launches(b);
  if (launches == 0) return HVX_SUCCESS;  // nothing to launch
  // A graph pays off only for several launches (a replay costs more than one
  // plain launch), and the legacy null stream cannot be captured at all.
  if (b->use_graph && s != nullptr && launches > 1) {
    if (!b->exec) {
      // capture once: the batch launch plus the launches of any graph
      // that is not expressible as batch work items
      hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) return set_error(b->ctx, HVX_ERROR_DEVICE, "begin capture: %s", hipGetErrorString(e));
      st = batch_enqueue(b, s);
      hipGraph_t hg = nullptr;
      e = hipStreamEndCapture(s, &hg);
      if (st) {
        if (hg) (void)hipGraphDestroy(hg);
        return st;
      }
      if (e != hipSuccess) return set_error(b->ctx, HVX_ERROR_DEVICE, "end capture: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&b->exec, hg, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(hg);
        b->exec = nullptr;
        return set_error(b->ctx, HVX_ERROR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
      }
      b->hg = hg;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return set_error(b->ctx, HVX_ERROR_DEVICE, "graph launch: %s", hipGetErrorString(e));
  } else {
    st = batch_enqueue(b, s);
    if (st) return st;
  }
  b->last_stream = stream;
  b->scheduled = true;
  return HVX_SUCCESS;
}

hvx_status hvx_batch_query(hvx_batch hb, int attr, int64_t* out) {
  if (!registry_check(hb, T_BATCH)) return HVX_ERROR_INVALID_REFERENCE;
  Batch* b = (Batch*)hb;
  if (!out) return set_error(b->ctx, HVX_ERROR_INVALID_PARAMETERS, "null output");
  switch (attr) {
    case HVX_QUERY_ALG_BYTES: *out = b->alg_bytes; break;
    case HVX_QUERY_NUM_KERNELS: *out = batch_launches(b); break;
    case HVX_QUERY_NUM_OPS: *out = b->total; break;  // work items of the single batch launch
    case HVX_QUERY_ROWS_PER_ITEM: *out = b->rows_override; break;  // 0: each graph's own
    default: return set_error(b->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown batch query %d", attr);
  }
  return HVX_SUCCESS;
}

// Outputs of the first and last graph of a batch (the tuner's equality check).
static hvx_status read_outputs(Graph* g, hipStream_t st, std::vector<std::vector<uint8_t>>* out);

// Rows per work item that make the single launch a whole number of rounds
// of resident waves (2, 3, 4, 6 or 8 rounds): the smallest rows whose item
// count fits, so the last round is as full as the batch allows.
static std::vector<int> balanced_rows(const Batch* b) {
  std::vector<std::pair<int64_t, int64_t>> sh;  // strips and height of each image
  for (const BatchImage& bi : b->imgs) {
    const StripGrid& g = bi.kind == FK_EDGE ? bi.d.e.g : bi.kind == FK_CORNER ? bi.d.c.g : bi.d.g5.g;
    sh.push_back({g.nstrips, g.h});
  }
  std::vector<int> out;
  if (sh.empty()) return out;
  const int64_t slots = (int64_t)b->ctx->num_cus * batch_waves_per_cu(b->kinds);
  auto items = [&](int64_t r) {
    int64_t n = 0;
    for (const auto& x : sh) n += x.first * ((x.second + r - 1) / r);
    return n;
  };
  for (int rounds : {2, 3, 4, 6, 8}) {
    const int64_t cap = rounds * slots;
    if (items(65535) > cap) continue;
    int lo = 1, hi = 65535;  // items() does not increase with the rows
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (items(mid) <= cap) hi = mid;
      else lo = mid + 1;
    }
    out.push_back(lo);
  }
  return out;
}

hvx_status hvx_batch_autotune(hvx_batch hb, void* stream, int iters) {
  if (!registry_check(hb, T_BATCH)) return HVX_ERROR_INVALID_REFERENCE;
  Batch* b = (Batch*)hb;
  if (iters < 1) iters = 1;
  hipStream_t st = (hipStream_t)stream;
  const bool saved_graph = b->use_graph;
  b->use_graph = false;  // time plain launches while candidates change
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  std::vector<std::vector<uint8_t>> ref, cur;
  double best = 1e30;
  int best_rows = b->rows_override;
  bool best_persistent = b->persistent;
  hvx_status s = HVX_SUCCESS;
  std::vector<int> cand_rows = {0, 8, 16, 24, 32, 40, 48, 64, 128};
  for (int r : balanced_rows(b))
    if (std::find(cand_rows.begin(), cand_rows.end(), r) == cand_rows.end()) cand_rows.push_back(r);
  for (int rows : cand_rows) {
    b->rows_override = rows;
    s = batch_build(b);
    if (s) break;
    for (int pers = 0; pers <= 1 && !s; ++pers) {
      b->persistent = pers != 0;
      s = batch_enqueue(b, st);
      if (!s && hipStreamSynchronize(st) != hipSuccess) s = set_error(b->ctx, HVX_ERROR_DEVICE, "tune sync failed");
      if (s) break;
      for (Graph* g : {b->graphs.front(), b->graphs.back()}) {
        std::vector<std::vector<uint8_t>> o;
        s = read_outputs(g, st, &o);
        if (s) break;
        for (auto& x : o) cur.push_back(std::move(x));
      }
      if (s) break;
      if (ref.empty()) {
        ref.swap(cur);
      } else if (cur != ref) {
        // name the first differing output byte and how many differ
        size_t which = 0, first = 0, count = 0;
        for (size_t i = 0; i < ref.size() && i < cur.size(); ++i) {
          if (ref[i] == cur[i]) continue;
          for (size_t j = 0; j < ref[i].size() && j < cur[i].size(); ++j) {
            if (ref[i][j] == cur[i][j]) continue;
            if (count == 0) {
              which = i;
              first = j;
            }
            ++count;
          }
        }
        s = set_error(b->ctx, HVX_ERROR_DEVICE,
                      "batch candidate rows=%d persistent=%d changed the output: %zu bytes differ, first in output "
                      "%zu at byte %zu (%u instead of %u)",
                      rows, pers, count, which, first, count ? (unsigned)cur[which][first] : 0u,
                      count ? (unsigned)ref[which][first] : 0u);
      }
      cur.clear();
      if (s) break;
      (void)hipEventRecord(e0, st);
      for (int i = 0; i < iters && !s; ++i) s = batch_enqueue(b, st);
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms / iters < best) {
        best = ms / iters;
        best_rows = rows;
        best_persistent = b->persistent;
      }
    }
    if (s) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->rows_override = best_rows;
  b->persistent = best_persistent;
  b->use_graph = saved_graph;
  hvx_status s2 = batch_build(b);
  return s ? s : s2;
}

hvx_status hvx_batch_set_option(hvx_batch hb, int option, int64_t value) {
  if (!registry_check(hb, T_BATCH)) return HVX_ERROR_INVALID_REFERENCE;
  Batch* b = (Batch*)hb;
  if (b->scheduled) (void)hipStreamSynchronize((hipStream_t)b->last_stream);
  b->scheduled = false;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->hg) (void)hipGraphDestroy(b->hg);
  b->exec = nullptr;
  b->hg = nullptr;
  switch (option) {
    case HVX_BATCH_PERSISTENT: b->persistent = value != 0; break;
    case HVX_BATCH_USE_GRAPH: b->use_graph = value != 0; break;
    case HVX_BATCH_ROWS:
      if (value < 0 || value > 65535) return set_error(b->ctx, HVX_ERROR_INVALID_PARAMETERS, "rows %lld", (long long)value);
      b->rows_override = (int)value;
      return batch_build(b);
    default: return set_error(b->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown batch option %d", option);
  }
  return HVX_SUCCESS;
}

hvx_status hvx_release_batch(hvx_batch* pb) {
  if (!pb || !registry_check(*pb, T_BATCH)) return HVX_ERROR_INVALID_REFERENCE;
  Batch* b = (Batch*)*pb;
  Context* c = b->ctx;
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    auto& v = c->children;
    v.erase(std::remove(v.begin(), v.end(), (Object*)b), v.end());
  }
  destroy_batch_object(b);
  *pb = nullptr;
  return HVX_SUCCESS;
}

hvx_status hvx_process_batch(hvx_context ctx, const hvx_graph* graphs, uint32_t n, void* stream) {
  hvx_batch b = nullptr;
  hvx_status s = hvx_batch_create(ctx, graphs, n, &b);
  if (s) return s;
  ((Batch*)b)->use_graph = false;
  s = hvx_batch_schedule(b, stream);
  if (!s && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    s = set_error((Context*)ctx, HVX_ERROR_DEVICE, "stream synchronize failed");
  hvx_release_batch(&b);
  return s;
}

// ---- autotuning -----------------------------------------------------------------

static hvx_status read_outputs(Graph* g, hipStream_t st, std::vector<std::vector<uint8_t>>* out) {
  // Copies ordered after the work on `st` and complete before returning.
  // The destination of the device-to-host copy is memory allocated pinned
  // (hipHostMalloc), then copied into the vector on the host: an
  // asynchronous copy into pageable memory makes the runtime pin or stage
  // the caller's pages on the fly, and where pinning memory that already
  // exists is refused, that copy can complete without writing the
  // destination (the comparison then sees the vector's zeros).
  out->clear();
  const Plan& p = *g->plan;
  for (size_t v = 0; v < p.vals.size(); ++v) {
    const Value& val = p.vals[v];
    if (val.is_virtual || val.producer < 0 || !p.ops[val.producer].live) continue;
    size_t row = (size_t)val.w * df_bytes(val.df);
    if (val.df == DF_BUF) {
      // a global operator's result: the words it defines (the rest of the
      // buffer is the reduction's workspace, whose contents depend on the
      // launch shape; location lists come in the order pixels were found)
      const LOp& op = p.ops[val.producer];
      switch (op.kind) {
        case OP_HISTOGRAM: row = (size_t)op.gp[0] * 4; break;
        case OP_MINMAX: row = kMinMaxBytes; break;
        case OP_MMCOUNT: row = 6 * 4; break;
        case OP_SUMS: row = kSumsBytes; break;
        default: continue;
      }
    }
    const size_t bytes = row * val.h;
    void* stage = nullptr;
    if (hipHostMalloc(&stage, bytes, 0) != hipSuccess)
      return set_error(g->ctx, HVX_ERROR_NO_MEMORY, "autotune readback: cannot allocate %zu pinned bytes", bytes);
    hipError_t e = hipMemcpy2DAsync(stage, row, val.img->ptr, val.img->pitch, row, val.h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) out->emplace_back((const uint8_t*)stage, (const uint8_t*)stage + bytes);
    (void)hipHostFree(stage);
    if (e != hipSuccess) return set_error(g->ctx, HVX_ERROR_DEVICE, "autotune readback: %s", hipGetErrorString(e));
  }
  return HVX_SUCCESS;
}

// Time `iters` schedules of the graph as planned now, after one checked
// run: its outputs must equal `ref` (or become `ref` when it is empty).
static hvx_status time_plan(Graph* g, hipStream_t st, int iters, std::vector<std::vector<uint8_t>>* ref,
                            double* us, const char* what) {
  hvx_status s = schedule_graph(g, st);
  if (!s && hipStreamSynchronize(st) != hipSuccess) s = set_error(g->ctx, HVX_ERROR_DEVICE, "tune sync failed");
  std::vector<std::vector<uint8_t>> cur;
  if (!s) s = read_outputs(g, st, ref->empty() ? ref : &cur);
  if (!s && !cur.empty() && cur != *ref) s = set_error(g->ctx, HVX_ERROR_DEVICE, "tune candidate %s changed the output", what);
  if (s) return s;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(e0, st);
  for (int i = 0; i < iters && !s; ++i) s = schedule_graph(g, st);
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *us = 1000.0 * ms / iters;
  return s;
}

// Re-plan the graph under plan choice `c` (null: none) and prepare it.
static hvx_status replan(Graph* g, const TuneEntry* c) {
  free_graph_device(g);
  g->plan_choice = c;
  hvx_status s = verify_graph(g);
  g->plan_choice = nullptr;
  if (!s) s = prepare_graph(g);
  return s;
}

// Plan choices (Section 6.3: whether fusing pays off depends on the
// operators and the device): the fused plan, every plan that cuts fusion at
// one value inside a fused group, and the plan that cuts at all of them;
// then, for the fastest, the tile of each generated group.  Every candidate
// must reproduce the outputs of the first one bit for bit.
static hvx_status tune_plan(Graph* g, hipStream_t st, int iters, std::vector<std::vector<uint8_t>>* ref,
                            TuneEntry* best) {
  const Plan& p0 = *g->plan;
  std::vector<int> internal;
  for (const Group& gr : p0.groups) {
    if (gr.ops.size() < 2) continue;
    std::set<int> ops(gr.ops.begin(), gr.ops.end());
    for (int o : gr.ops) {
      const int v = p0.ops[o].out;
      bool inside = false;
      for (int c : p0.vals[v].consumers) inside |= ops.count(c) > 0;
      if (inside) internal.push_back(v);
    }
  }
  std::vector<TuneEntry> cands(1);
  if (g->opt_fusion && !internal.empty()) {
    for (int v : internal) {
      cands.emplace_back();
      cands.back().cuts = {v};
    }
    if (internal.size() > 1) {
      cands.emplace_back();
      cands.back().cuts = internal;
    }
  }
  hvx_status s = HVX_SUCCESS;
  best->us = 1e30;
  for (TuneEntry& c : cands) {
    c.has_plan = true;
    double us = 0;
    s = replan(g, &c);
    if (!s) s = time_plan(g, st, iters, ref, &us, "plan");
    if (s) return s;
    if (us < best->us) {
      *best = c;
      best->us = us;
    }
  }
  // tiles of the generated groups of the chosen plan, one group at a time
  s = replan(g, best);
  if (s) return s;
  std::vector<int> firsts;
  for (const auto& t : g->plan->tiles) firsts.push_back(t[0]);
  static const int shapes[][2] = {{128, 16}, {64, 16}, {64, 32}, {128, 8}, {256, 8}, {32, 16}};
  for (int first : firsts) {
    for (auto& sh : shapes) {
      TuneEntry c = *best;
      bool found = false;
      for (auto& t : c.tiles)
        if (t[0] == first) {
          t[1] = sh[0];
          t[2] = sh[1];
          found = true;
        }
      if (!found) c.tiles.push_back({first, sh[0], sh[1]});
      double us = 0;
      s = replan(g, &c);
      if (s) return s;
      bool applied = false;  // the shape fits the group's LDS budget
      for (const auto& t : g->plan->tiles) applied |= t[0] == first && t[1] == sh[0] && t[2] == sh[1];
      if (!applied) continue;
      s = time_plan(g, st, iters, ref, &us, "tile");
      if (s) return s;
      if (us < best->us) {
        *best = c;
        best->us = us;
      }
    }
  }
  return HVX_SUCCESS;
}

hvx_status hvx_graph_autotune(hvx_graph hg, void* stream, int iters) {
  if (!registry_check(hg, T_GRAPH)) return HVX_ERROR_INVALID_REFERENCE;
  Graph* g = (Graph*)hg;
  std::lock_guard<std::recursive_mutex> lock(g->ctx->mu);
  if (iters < 1) iters = 1;
  hipStream_t st = (hipStream_t)stream;
  // the outputs of the plan in force before tuning: every candidate must reproduce them
  std::vector<std::vector<uint8_t>> ref;
  hvx_status s = replan(g, nullptr);
  double us0 = 0;
  if (!s) s = time_plan(g, st, 1, &ref, &us0, "default");
  if (s) return s;
  TuneEntry plan;
  s = tune_plan(g, st, iters, &ref, &plan);
  if (!s) {
    g->ctx->tune["plan|" + g->plan->op_key] = plan;
    s = replan(g, nullptr);  // the graph runs the recorded choice from here on
  }
  if (s) return s;
  Plan& p = *g->plan;
  if (p.groups.size() != 1 || !is_strip_kind(p.groups[0].kind)) return HVX_SUCCESS;  // no launch shape to tune
  // rows per work item and the XCD mapping of a hand-fused kernel
  Group& gr = p.groups[0];
  const int saved_rows = gr.rows, saved_xcd = gr.xcd;
  double best_us = 1e30;
  int best_rows = 0, best_xcd = 1;
  static const int cand_rows[] = {4, 8, 16, 32, 64, 128};
  for (int rows : cand_rows) {
    if (rows > (int)gr.h * 2 && rows != 4) continue;
    for (int xcd = 0; xcd <= 1 && !s; ++xcd) {
      gr.rows = rows;
      gr.xcd = xcd;
      double us = 0;
      char what[48];
      snprintf(what, sizeof what, "rows=%d xcd=%d", rows, xcd);
      s = time_plan(g, st, iters, &ref, &us, what);
      if (!s && us < best_us) {
        best_us = us;
        best_rows = rows;
        best_xcd = xcd;
      }
    }
    if (s) break;
  }
  gr.rows = saved_rows;
  gr.xcd = saved_xcd;
  if (s) return s;
  TuneEntry t;
  t.rows = best_rows;
  t.xcd = best_xcd;
  t.us = best_us;
  g->ctx->tune[tune_key(g)] = t;
  return HVX_SUCCESS;
}

// Tune cache file: one JSON object, {"key": [rows, xcd, microseconds], ...}; a plan
// choice adds its cut values and generated tiles: [..., [cuts], [[first, w, h], ...]].
hvx_status hvx_context_save_tune_cache(hvx_context ctx, const char* path) {
  if (!registry_check(ctx, T_CONTEXT)) return HVX_ERROR_INVALID_REFERENCE;
  Context* c = (Context*)ctx;
  if (!path) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null path");
  std::ofstream f(path);
  if (!f) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "cannot write %s", path);
  f << "{";
  bool first = true;
  for (auto& kv : c->tune) {
    std::string k;
    for (char ch : kv.first) {
      if (ch == '"' || ch == '\\') k += '\\';
      k += ch;
    }
    const TuneEntry& e = kv.second;
    f << (first ? "" : ",") << "\n  \"" << k << "\": [" << e.rows << ", " << e.xcd << ", " << e.us;
    if (e.has_plan) {  // plan choice: [cut values], [[first operator, tile width, tile height], ...]
      f << ", [";
      for (size_t i = 0; i < e.cuts.size(); ++i) f << (i ? ", " : "") << e.cuts[i];
      f << "], [";
      for (size_t i = 0; i < e.tiles.size(); ++i)
        f << (i ? ", " : "") << "[" << e.tiles[i][0] << ", " << e.tiles[i][1] << ", " << e.tiles[i][2] << "]";
      f << "]";
    }
    f << "]";
    first = false;
  }
  f << "\n}\n";
  return f.good() ? HVX_SUCCESS : set_error(c, HVX_ERROR_INVALID_PARAMETERS, "write failed");
}

hvx_status hvx_context_load_tune_cache(hvx_context ctx, const char* path) {
  if (!registry_check(ctx, T_CONTEXT)) return HVX_ERROR_INVALID_REFERENCE;
  Context* c = (Context*)ctx;
  if (!path) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null path");
  std::ifstream f(path);
  if (!f) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "cannot read %s", path);
  std::stringstream ss;
  ss << f.rdbuf();
  std::string t = ss.str();
  size_t i = 0;
  int n = 0;
  while (true) {
    size_t q = t.find('"', i);
    if (q == std::string::npos) break;
    std::string key;
    size_t j = q + 1;
    for (; j < t.size() && t[j] != '"'; ++j) {
      if (t[j] == '\\' && j + 1 < t.size()) ++j;
      key += t[j];
    }
    // the entry's list, brackets matched: [rows, xcd, us] or, for a plan
    // choice, [rows, xcd, us, [cuts], [[first, width, height], ...]]
    size_t lb = t.find('[', j), rb = std::string::npos;
    int depth = 0;
    for (size_t z = lb; lb != std::string::npos && z < t.size(); ++z) {
      if (t[z] == '[') ++depth;
      if (t[z] == ']' && --depth == 0) {
        rb = z;
        break;
      }
    }
    if (lb == std::string::npos || rb == std::string::npos)
      return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "malformed tune cache %s", path);
    TuneEntry e;
    if (sscanf(t.c_str() + lb + 1, "%d , %d , %lf", &e.rows, &e.xcd, &e.us) != 3)
      return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "malformed tune entry for %s", key.c_str());
    const size_t inner = t.find('[', lb + 1);
    if (inner != std::string::npos && inner < rb) {
      // numbers of the two inner lists, in order
      std::vector<std::vector<int>> lists(1);
      int d = 0;
      for (size_t z = inner; z < rb; ++z) {
        if (t[z] == '[') ++d;
        else if (t[z] == ']') {
          if (--d == 0) lists.emplace_back();
        } else if (t[z] == '-' || (t[z] >= '0' && t[z] <= '9')) {
          char* end = nullptr;
          lists.back().push_back((int)strtol(t.c_str() + z, &end, 10));
          z = (size_t)(end - t.c_str()) - 1;
        }
      }
      if (lists.size() < 3 || lists[1].size() % 3 != 0)
        return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "malformed plan choice for %s", key.c_str());
      e.has_plan = true;
      e.cuts = lists[0];
      for (size_t q = 0; q + 2 < lists[1].size(); q += 3) e.tiles.push_back({lists[1][q], lists[1][q + 1], lists[1][q + 2]});
    }
    c->tune[key] = e;
    ++n;
    i = rb + 1;
  }
  return HVX_SUCCESS;
}

}  // extern "C"
