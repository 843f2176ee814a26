// C ABI of the hvx library: objects, node constructors, release, queries.
// The graph formulation follows OpenVX as used in Section 3.1 of the paper:
// objects live in a context, nodes connect (virtual) images, and a graph is
// verified before it is processed.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "global.h"
#include "hvx_internal.h"

namespace hvx {

// ---- handle registry: a released or foreign handle is detected, not used --
static std::mutex g_reg_mu;
static std::unordered_map<const void*, uint32_t>& reg() {
  static std::unordered_map<const void*, uint32_t> m;
  return m;
}

bool registry_check(const void* h, uint32_t type) {
  if (!h) return false;
  std::lock_guard<std::mutex> l(g_reg_mu);
  auto it = reg().find(h);
  return it != reg().end() && it->second == type;
}
void registry_add(Object* o) {
  std::lock_guard<std::mutex> l(g_reg_mu);
  reg()[o] = o->type;
}
void registry_remove(Object* o) {
  std::lock_guard<std::mutex> l(g_reg_mu);
  reg().erase(o);
}

hvx_status set_error(Context* ctx, hvx_status s, const char* fmt, ...) {
  if (ctx && s != HVX_SUCCESS) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::lock_guard<std::recursive_mutex> l(ctx->mu);
    ctx->last_error = buf;
  }
  return s;
}

template <class T>
static T* as(const void* h, uint32_t type) {
  return registry_check(h, type) ? (T*)h : nullptr;
}

static void remove_child(Context* c, Object* o) {
  std::lock_guard<std::recursive_mutex> l(c->mu);
  auto& v = c->children;
  v.erase(std::remove(v.begin(), v.end(), o), v.end());
}

static void destroy_image(Image* im) {
  if (im->owned && im->ptr) (void)hipFree(im->ptr);
  im->ptr = nullptr;
  registry_remove(im);
  delete im;
}

static void destroy_graph(Graph* g) {
  free_graph_device(g);
  for (Node* n : g->nodes) {
    registry_remove(n);
    delete n;
  }
  for (Image* v : g->virt) destroy_image(v);
  registry_remove(g);
  delete g;
}

static void invalidate(Graph* g) {
  if (g->verified) free_graph_device(g);
  g->verified = false;
  g->plan.reset();
}

}  // namespace hvx

using namespace hvx;

// batch and server objects are destroyed from their own translation units
namespace hvx {
void destroy_batch_object(Object* o);
void destroy_server_object(Object* o);
}  // namespace hvx

extern "C" {

const char* hvx_status_name(hvx_status s) {
  switch (s) {
    case HVX_SUCCESS: return "HVX_SUCCESS";
    case HVX_ERROR_INVALID_REFERENCE: return "HVX_ERROR_INVALID_REFERENCE";
    case HVX_ERROR_INVALID_PARAMETERS: return "HVX_ERROR_INVALID_PARAMETERS";
    case HVX_ERROR_INVALID_FORMAT: return "HVX_ERROR_INVALID_FORMAT";
    case HVX_ERROR_INVALID_DIMENSION: return "HVX_ERROR_INVALID_DIMENSION";
    case HVX_ERROR_INVALID_GRAPH: return "HVX_ERROR_INVALID_GRAPH";
    case HVX_ERROR_NOT_VERIFIED: return "HVX_ERROR_NOT_VERIFIED";
    case HVX_ERROR_NO_MEMORY: return "HVX_ERROR_NO_MEMORY";
    case HVX_ERROR_NOT_SUPPORTED: return "HVX_ERROR_NOT_SUPPORTED";
    case HVX_ERROR_DEVICE: return "HVX_ERROR_DEVICE";
    default: return "HVX_UNKNOWN_STATUS";
  }
}

hvx_status hvx_context_create(int hip_device, hvx_context* out) {
  if (!out) return HVX_ERROR_INVALID_PARAMETERS;
  *out = nullptr;
  if (hip_device < 0) return HVX_ERROR_INVALID_PARAMETERS;
  Context* c = new (std::nothrow) Context();
  if (!c) return HVX_ERROR_NO_MEMORY;
  c->type = T_CONTEXT;
  c->ctx = c;
  c->device = hip_device;
  registry_add(c);
  *out = (hvx_context)c;
  return HVX_SUCCESS;
}

hvx_status hvx_context_release(hvx_context* pctx) {
  if (!pctx) return HVX_ERROR_INVALID_PARAMETERS;
  Context* c = as<Context>(*pctx, T_CONTEXT);
  if (!c) return HVX_ERROR_INVALID_REFERENCE;
  if (c->dev_ready) {
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
  }
  std::vector<Object*> kids;
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    kids.swap(c->children);
  }
  // servers and batches first (they reference graphs), then graphs, then the rest
  for (Object* o : kids)
    if (o->type == T_SERVER) destroy_server_object(o);
  for (Object* o : kids)
    if (o->type == T_BATCH) destroy_batch_object(o);
  for (Object* o : kids)
    if (o->type == T_GRAPH) destroy_graph((Graph*)o);
  for (Object* o : kids) {
    if (o->type == T_IMAGE || o->type == T_BUFFER) destroy_image((Image*)o);
    else if (o->type == T_CONV || o->type == T_NODE) {
      registry_remove(o);
      delete o;
    }
  }
  registry_remove(c);
  delete c;
  *pctx = nullptr;
  return HVX_SUCCESS;
}

const char* hvx_last_error(hvx_context ctx) {
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!c) return "invalid context";
  std::lock_guard<std::recursive_mutex> l(c->mu);
  return c->last_error.c_str();
}

// ---- images ----------------------------------------------------------------

static bool valid_df(int df) { return df >= DF_U8 && df <= DF_UYVY; }

static hvx_status check_layout(Context* c, uint32_t w, uint32_t h, int df, void* ptr, size_t pitch) {
  if (!valid_df(df)) return set_error(c, HVX_ERROR_INVALID_FORMAT, "unknown image format %d", df);
  if (w == 0 || h == 0 || w > 65536 || h > 65536)
    return set_error(c, HVX_ERROR_INVALID_DIMENSION, "image size %ux%u out of range", w, h);
  if (df == DF_UYVY && (w & 1)) return set_error(c, HVX_ERROR_INVALID_DIMENSION, "UYVY width must be even");
  if (!ptr) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null device pointer");
  if (pitch % 64 != 0 || pitch < (size_t)w * df_bytes(df))
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "pitch %zu must be a multiple of 64 and >= %zu", pitch,
                     (size_t)w * df_bytes(df));
  if (((uintptr_t)ptr) % 16 != 0)
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "device pointer must be 16-byte aligned");
  return HVX_SUCCESS;
}

hvx_status hvx_image_from_ptr(hvx_context ctx, uint32_t w, uint32_t h, int df, void* ptr, size_t pitch,
                              hvx_image* out) {
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!c) return HVX_ERROR_INVALID_REFERENCE;
  if (!out) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null output handle");
  *out = nullptr;
  hvx_status s = check_layout(c, w, h, df, ptr, pitch);
  if (s) return s;
  Image* im = new Image();
  im->type = T_IMAGE;
  im->ctx = c;
  im->w = w;
  im->h = h;
  im->df = df;
  im->ptr = ptr;
  im->pitch = pitch;
  registry_add(im);
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    c->children.push_back(im);
  }
  *out = (hvx_image)im;
  return HVX_SUCCESS;
}

hvx_status hvx_image_create(hvx_context ctx, uint32_t w, uint32_t h, int df, hvx_image* out) {
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!c) return HVX_ERROR_INVALID_REFERENCE;
  if (!out) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null output handle");
  *out = nullptr;
  if (!valid_df(df)) return set_error(c, HVX_ERROR_INVALID_FORMAT, "unknown image format %d", df);
  if (w == 0 || h == 0 || w > 65536 || h > 65536)
    return set_error(c, HVX_ERROR_INVALID_DIMENSION, "image size %ux%u out of range", w, h);
  hvx_status s = ensure_device(c);
  if (s) return s;
  size_t pitch = ((size_t)w * df_bytes(df) + 63) / 64 * 64;
  void* p = nullptr;
  if (hipMalloc(&p, pitch * h) != hipSuccess)
    return set_error(c, HVX_ERROR_NO_MEMORY, "hipMalloc of %zu bytes failed", pitch * h);
  hvx_image im = nullptr;
  s = hvx_image_from_ptr(ctx, w, h, df, p, pitch, &im);
  if (s) {
    (void)hipFree(p);
    return s;
  }
  ((Image*)im)->owned = true;
  *out = im;
  return HVX_SUCCESS;
}

hvx_status hvx_image_swap_ptr(hvx_image img, void* ptr, size_t pitch) {
  Image* im = as<Image>(img, T_IMAGE);
  if (!im) return HVX_ERROR_INVALID_REFERENCE;
  if (im->is_virtual) return set_error(im->ctx, HVX_ERROR_INVALID_PARAMETERS, "virtual images have no pointer");
  if (im->owned) return set_error(im->ctx, HVX_ERROR_INVALID_PARAMETERS, "library-owned image");
  hvx_status s = check_layout(im->ctx, im->w, im->h, im->df, ptr, pitch);
  if (s) return s;
  im->ptr = ptr;
  im->pitch = pitch;
  return HVX_SUCCESS;
}

hvx_status hvx_image_query(hvx_image img, uint32_t* w, uint32_t* h, int* df, void** ptr, size_t* pitch) {
  Image* im = as<Image>(img, T_IMAGE);
  if (!im) return HVX_ERROR_INVALID_REFERENCE;
  if (w) *w = im->w;
  if (h) *h = im->h;
  if (df) *df = im->df;
  if (ptr) *ptr = im->is_virtual ? nullptr : im->ptr;
  if (pitch) *pitch = im->is_virtual ? 0 : im->pitch;
  return HVX_SUCCESS;
}

hvx_status hvx_image_copy(hvx_image img, void* host, size_t host_pitch, int to_device) {
  Image* im = as<Image>(img, T_IMAGE);
  if (!im) return HVX_ERROR_INVALID_REFERENCE;
  Context* c = im->ctx;
  if (im->is_virtual) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "virtual images are not accessible");
  size_t row = (size_t)im->w * df_bytes(im->df);
  if (!host || host_pitch < row) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "bad host buffer or pitch");
  hvx_status s = ensure_device(c);
  if (s) return s;
  hipError_t e = to_device ? hipMemcpy2D(im->ptr, im->pitch, host, host_pitch, row, im->h, hipMemcpyHostToDevice)
                           : hipMemcpy2D(host, host_pitch, im->ptr, im->pitch, row, im->h, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return set_error(c, HVX_ERROR_DEVICE, "hipMemcpy2D: %s", hipGetErrorString(e));
  return HVX_SUCCESS;
}

hvx_status hvx_image_create_virtual(hvx_graph graph, uint32_t w, uint32_t h, int df, hvx_image* out) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  if (!out) return set_error(g->ctx, HVX_ERROR_INVALID_PARAMETERS, "null output handle");
  *out = nullptr;
  if (df != DF_VIRT && !valid_df(df)) return set_error(g->ctx, HVX_ERROR_INVALID_FORMAT, "unknown format %d", df);
  if ((w == 0) != (h == 0))
    return set_error(g->ctx, HVX_ERROR_INVALID_DIMENSION, "give both or neither of width and height");
  Image* im = new Image();
  im->type = T_IMAGE;
  im->ctx = g->ctx;
  im->w = w;
  im->h = h;
  im->df = df;
  im->is_virtual = true;
  im->vgraph = g;
  registry_add(im);
  g->virt.push_back(im);
  invalidate(g);
  *out = (hvx_image)im;
  return HVX_SUCCESS;
}

hvx_status hvx_convolution_create(hvx_context ctx, uint32_t cols, uint32_t rows, const int16_t* coeffs,
                                  uint32_t scale, hvx_convolution* out) {
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!c) return HVX_ERROR_INVALID_REFERENCE;
  if (!out || !coeffs) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null argument");
  *out = nullptr;
  if (cols < 1 || rows < 1 || cols > 5 || rows > 5 || !(cols & 1) || !(rows & 1))
    return set_error(c, HVX_ERROR_INVALID_DIMENSION, "mask must be odd-sized, at most 5x5 (got %ux%u)", cols, rows);
  if (scale == 0 || (scale & (scale - 1)) || scale > 32768)
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "scale %u is not a power of two in [1, 2^15]", scale);
  Conv* cv = new Conv();
  cv->type = T_CONV;
  cv->ctx = c;
  cv->cols = cols;
  cv->rows = rows;
  cv->scale = scale;
  cv->coeffs.assign(coeffs, coeffs + cols * rows);
  registry_add(cv);
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    c->children.push_back(cv);
  }
  *out = (hvx_convolution)cv;
  return HVX_SUCCESS;
}

hvx_status hvx_buffer_from_ptr(hvx_context ctx, void* dev_ptr, size_t bytes, hvx_buffer* out) {
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!c) return HVX_ERROR_INVALID_REFERENCE;
  if (!out) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null output handle");
  *out = nullptr;
  if (!dev_ptr || ((uintptr_t)dev_ptr & 7))
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "buffer pointer null or not 8-byte aligned");
  if (bytes == 0 || bytes > ((size_t)1 << 31))
    return set_error(c, HVX_ERROR_INVALID_DIMENSION, "buffer size %zu out of range", bytes);
  Image* b = new Image();
  b->type = T_BUFFER;
  b->ctx = c;
  b->w = (uint32_t)bytes;
  b->h = 1;
  b->df = DF_BUF;
  b->ptr = dev_ptr;
  b->pitch = bytes;
  registry_add(b);
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    c->children.push_back(b);
  }
  *out = (hvx_buffer)b;
  return HVX_SUCCESS;
}

// ---- graph and nodes -------------------------------------------------------

hvx_status hvx_graph_create(hvx_context ctx, hvx_graph* out) {
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!c) return HVX_ERROR_INVALID_REFERENCE;
  if (!out) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null output handle");
  Graph* g = new Graph();
  g->type = T_GRAPH;
  g->ctx = c;
  registry_add(g);
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    c->children.push_back(g);
  }
  *out = (hvx_graph)g;
  return HVX_SUCCESS;
}

// Shared constructor: presence checks only; formats and sizes at verify.
static hvx_status add_node(hvx_graph graph, int kind, std::initializer_list<hvx_image> ins,
                           std::initializer_list<hvx_image> outs, int min_outs, hvx_node* node_out, Node** made) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  if (node_out) *node_out = nullptr;
  for (hvx_image i : ins)
    if (!registry_check(i, T_IMAGE)) return set_error(g->ctx, HVX_ERROR_INVALID_REFERENCE, "invalid input image");
  int present = 0;
  for (hvx_image o : outs) {
    if (!o) continue;
    if (!registry_check(o, T_IMAGE)) return set_error(g->ctx, HVX_ERROR_INVALID_REFERENCE, "invalid output image");
    ++present;
  }
  if (present < min_outs) return set_error(g->ctx, HVX_ERROR_INVALID_PARAMETERS, "missing output image");
  for (hvx_image i : ins)
    if (((Image*)i)->ctx != g->ctx)
      return set_error(g->ctx, HVX_ERROR_INVALID_GRAPH, "input image belongs to another context");
  for (hvx_image o : outs)
    if (o && ((Image*)o)->ctx != g->ctx)
      return set_error(g->ctx, HVX_ERROR_INVALID_GRAPH, "output image belongs to another context");
  Node* n = new Node();
  n->type = T_NODE;
  n->ctx = g->ctx;
  n->g = g;
  n->kind = kind;
  for (hvx_image i : ins) n->in.push_back((Image*)i);
  for (hvx_image o : outs) n->out.push_back((Image*)o);
  registry_add(n);
  g->nodes.push_back(n);
  invalidate(g);
  if (node_out) *node_out = (hvx_node)n;
  if (made) *made = n;
  return HVX_SUCCESS;
}

hvx_status hvx_channel_extract_node(hvx_graph g, hvx_image uyvy, int channel, hvx_image out, hvx_node* no) {
  if (channel != HVX_CHANNEL_Y) {
    Graph* gg = as<Graph>(g, T_GRAPH);
    return gg ? set_error(gg->ctx, HVX_ERROR_NOT_SUPPORTED, "only the Y channel of UYVY is supported")
              : HVX_ERROR_INVALID_REFERENCE;
  }
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_CHANNEL_EXTRACT, {uyvy}, {out}, 1, no, &n);
  if (!s) n->channel = channel;
  return s;
}
hvx_status hvx_gaussian3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_GAUSS3, {in}, {out}, 1, no, nullptr);
}
hvx_status hvx_gaussian5x5_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_GAUSS5, {in}, {out}, 1, no, nullptr);
}
hvx_status hvx_box3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_BOX3, {in}, {out}, 1, no, nullptr);
}

hvx_status hvx_dilate3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_DILATE3, {in}, {out}, 1, no, nullptr);
}

hvx_status hvx_erode3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_ERODE3, {in}, {out}, 1, no, nullptr);
}

hvx_status hvx_median3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_MEDIAN3, {in}, {out}, 1, no, nullptr);
}
hvx_status hvx_box5x5_f32_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_BOX5F, {in}, {out}, 1, no, nullptr);
}
hvx_status hvx_sobel3x3_node(hvx_graph g, hvx_image in, hvx_image gx, hvx_image gy, hvx_node* no) {
  return add_node(g, NK_SOBEL3, {in}, {gx, gy}, 1, no, nullptr);
}
hvx_status hvx_magnitude_node(hvx_graph g, hvx_image gx, hvx_image gy, hvx_image out, hvx_node* no) {
  return add_node(g, NK_MAGNITUDE, {gx, gy}, {out}, 1, no, nullptr);
}
hvx_status hvx_phase_node(hvx_graph g, hvx_image gx, hvx_image gy, hvx_image out, hvx_node* no) {
  return add_node(g, NK_PHASE, {gx, gy}, {out}, 1, no, nullptr);
}
hvx_status hvx_add_node(hvx_graph g, hvx_image a, hvx_image b, int policy, hvx_image out, hvx_node* no) {
  if (policy != HVX_POLICY_SATURATE && policy != HVX_POLICY_WRAP) {
    Graph* gg = as<Graph>(g, T_GRAPH);
    return gg ? set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown overflow policy %d", policy)
              : HVX_ERROR_INVALID_REFERENCE;
  }
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_ADD, {a, b}, {out}, 1, no, &n);
  if (!s) n->policy = policy;
  return s;
}
hvx_status hvx_multiply_f32_node(hvx_graph g, hvx_image a, hvx_image b, hvx_image out, hvx_node* no) {
  return add_node(g, NK_MULF, {a, b}, {out}, 1, no, nullptr);
}
hvx_status hvx_harris_response_node(hvx_graph g, hvx_image sxx, hvx_image syy, hvx_image sxy, float k,
                                    hvx_image out, hvx_node* no) {
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_HARRIS, {sxx, syy, sxy}, {out}, 1, no, &n);
  if (!s) n->k = k;
  return s;
}
hvx_status hvx_threshold_node(hvx_graph g, hvx_image in, double value, uint8_t tv, uint8_t fv, hvx_image out,
                              hvx_node* no) {
  if (!(value == value)) {
    Graph* gg = as<Graph>(g, T_GRAPH);
    return gg ? set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "threshold is NaN") : HVX_ERROR_INVALID_REFERENCE;
  }
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_THRESHOLD, {in}, {out}, 1, no, &n);
  if (!s) {
    n->dval = value;
    n->tv = tv;
    n->fv = fv;
  }
  return s;
}
// Global operator nodes: one image in, result buffers out (a NULL buffer
// only where the call allows it).
static hvx_status add_global_node(hvx_graph graph, int kind, hvx_image in, std::initializer_list<hvx_buffer> outs,
                                  int min_outs, hvx_node* node_out, Node** made) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  if (node_out) *node_out = nullptr;
  if (!registry_check(in, T_IMAGE)) return set_error(g->ctx, HVX_ERROR_INVALID_REFERENCE, "invalid input image");
  if (((Image*)in)->ctx != g->ctx)
    return set_error(g->ctx, HVX_ERROR_INVALID_GRAPH, "input image belongs to another context");
  int present = 0;
  for (hvx_buffer b : outs) {
    if (!b) continue;
    if (!registry_check(b, T_BUFFER)) return set_error(g->ctx, HVX_ERROR_INVALID_REFERENCE, "invalid result buffer");
    if (((Image*)b)->ctx != g->ctx)
      return set_error(g->ctx, HVX_ERROR_INVALID_GRAPH, "result buffer belongs to another context");
    ++present;
  }
  if (present < min_outs) return set_error(g->ctx, HVX_ERROR_INVALID_PARAMETERS, "missing result buffer");
  Node* n = new Node();
  n->type = T_NODE;
  n->ctx = g->ctx;
  n->g = g;
  n->kind = kind;
  n->in.push_back((Image*)in);
  for (hvx_buffer b : outs) n->out.push_back((Image*)b);
  registry_add(n);
  g->nodes.push_back(n);
  invalidate(g);
  if (node_out) *node_out = (hvx_node)n;
  if (made) *made = n;
  return HVX_SUCCESS;
}

hvx_status hvx_histogram_node(hvx_graph g, hvx_image in, uint32_t num_bins, uint32_t offset, uint32_t range,
                              hvx_buffer counts, hvx_node* no) {
  Graph* gg = as<Graph>(g, T_GRAPH);
  if (!gg) return HVX_ERROR_INVALID_REFERENCE;
  if (num_bins < 1 || num_bins > 256 || range < num_bins || offset + (uint64_t)range > 256)
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "need 1 <= num_bins <= range and offset + range <= 256");
  Node* n = nullptr;
  hvx_status s = add_global_node(g, NK_HISTOGRAM, in, {counts}, 1, no, &n);
  if (!s) {
    n->gp[0] = num_bins;
    n->gp[1] = offset;
    n->gp[2] = range;
  }
  return s;
}
hvx_status hvx_min_max_node(hvx_graph g, hvx_image in, hvx_buffer result, hvx_node* no) {
  return add_global_node(g, NK_MINMAX, in, {result}, 1, no, nullptr);
}
hvx_status hvx_min_max_loc_node(hvx_graph g, hvx_image in, hvx_buffer result, hvx_buffer locations,
                                uint32_t capacity, hvx_node* no) {
  Graph* gg = as<Graph>(g, T_GRAPH);
  if (!gg) return HVX_ERROR_INVALID_REFERENCE;
  if ((capacity == 0) != (locations == nullptr))
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "locations and a capacity go together");
  if (capacity > (1u << 24)) return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "capacity above 2^24");
  Node* n = nullptr;
  hvx_status s = add_global_node(g, NK_MINMAXLOC, in, {result, locations}, 1, no, &n);
  if (!s) n->gp[0] = capacity;
  return s;
}
hvx_status hvx_mean_std_dev_node(hvx_graph g, hvx_image in, hvx_buffer result, hvx_node* no) {
  return add_global_node(g, NK_MEANSTD, in, {result}, 1, no, nullptr);
}
hvx_status hvx_equalize_hist_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* no) {
  return add_node(g, NK_EQHIST, {in}, {out}, 1, no, nullptr);
}

hvx_status hvx_convolve_node(hvx_graph g, hvx_image in, hvx_convolution conv, hvx_image out, hvx_node* no) {
  Graph* gg = as<Graph>(g, T_GRAPH);
  if (!gg) return HVX_ERROR_INVALID_REFERENCE;
  Conv* cv = as<Conv>(conv, T_CONV);
  if (!cv) return set_error(gg->ctx, HVX_ERROR_INVALID_REFERENCE, "invalid convolution");
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_CONVOLVE, {in}, {out}, 1, no, &n);
  if (!s) n->conv = cv;
  return s;
}

hvx_status hvx_nonlinear_filter_node(hvx_graph g, int function, hvx_image in, uint32_t cols, uint32_t rows,
                                     const uint8_t* mask, hvx_image out, hvx_node* no) {
  Graph* gg = as<Graph>(g, T_GRAPH);
  if (!gg) return HVX_ERROR_INVALID_REFERENCE;
  if (function < HVX_NONLINEAR_MEDIAN || function > HVX_NONLINEAR_MAX)
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown nonlinear function %d", function);
  if (cols < 1 || rows < 1 || cols > 5 || rows > 5 || !(cols & 1) || !(rows & 1))
    return set_error(gg->ctx, HVX_ERROR_INVALID_DIMENSION, "mask must be odd-sized, at most 5x5 (got %ux%u)", cols,
                     rows);
  if (!mask) return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "null mask");
  bool any = false;
  for (uint32_t k = 0; k < cols * rows; ++k) any |= mask[k] != 0;
  if (!any) return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "mask has no nonzero entry");
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_NONLINEAR, {in}, {out}, 1, no, &n);
  if (s) return s;
  n->policy = function;
  n->own_mask.type = T_CONV;
  n->own_mask.ctx = gg->ctx;
  n->own_mask.cols = cols;
  n->own_mask.rows = rows;
  n->own_mask.scale = 1;
  n->own_mask.coeffs.resize(cols * rows);
  for (uint32_t k = 0; k < cols * rows; ++k) n->own_mask.coeffs[k] = mask[k] != 0;
  n->conv = &n->own_mask;
  return HVX_SUCCESS;
}

hvx_status hvx_non_max_suppression_node(hvx_graph g, hvx_image in, uint32_t win_size, hvx_image out, hvx_node* no) {
  Graph* gg = as<Graph>(g, T_GRAPH);
  if (!gg) return HVX_ERROR_INVALID_REFERENCE;
  if (win_size != 3 && win_size != 5)
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "window size must be 3 or 5 (got %u)", win_size);
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_NONMAX, {in}, {out}, 1, no, &n);
  if (!s) n->policy = (int)win_size;
  return s;
}

hvx_status hvx_custom_point_node(hvx_graph g, const char* expr, const hvx_image* inputs, uint32_t num_inputs,
                                 int out_format, hvx_image out, hvx_node* no) {
  Graph* gg = as<Graph>(g, T_GRAPH);
  if (!gg) return HVX_ERROR_INVALID_REFERENCE;
  if (num_inputs < 1 || num_inputs > 3 || !inputs)
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "a user point kernel takes 1 to 3 inputs (got %u)",
                     num_inputs);
  if (out_format != HVX_DF_U8 && out_format != HVX_DF_S16 && out_format != HVX_DF_F32)
    return set_error(gg->ctx, HVX_ERROR_INVALID_FORMAT, "output format must be U8, S16 or F32");
  ExprProg prog;
  std::string why = parse_expr(expr, &prog);
  if (!why.empty()) return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "expression: %s", why.c_str());
  if (prog.max_input >= (int)num_inputs)
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "expression names input %c of %u", 'a' + prog.max_input,
                     num_inputs);
  if (prog.has_offsets)
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "window offsets need a user local kernel");
  Node* n = nullptr;
  hvx_status s = num_inputs == 1   ? add_node(g, NK_CUSTOM_POINT, {inputs[0]}, {out}, 1, no, &n)
                 : num_inputs == 2 ? add_node(g, NK_CUSTOM_POINT, {inputs[0], inputs[1]}, {out}, 1, no, &n)
                                   : add_node(g, NK_CUSTOM_POINT, {inputs[0], inputs[1], inputs[2]}, {out}, 1, no, &n);
  if (s) return s;
  n->expr = std::move(prog);
  n->out_df = out_format;
  return HVX_SUCCESS;
}

// ---- global operators (immediate mode) ------------------------------------------

static hvx_status global_input(hvx_context ctx, hvx_image in, std::initializer_list<int> dfs, GlobalImg* gi) {
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!c) return HVX_ERROR_INVALID_REFERENCE;
  Image* im = as<Image>(in, T_IMAGE);
  if (!im || im->ctx != c) return set_error(c, HVX_ERROR_INVALID_REFERENCE, "invalid image");
  if (im->is_virtual || !im->ptr) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "image has no device memory");
  bool ok = false;
  for (int d : dfs) ok |= im->df == d;
  if (!ok) return set_error(c, HVX_ERROR_INVALID_FORMAT, "unsupported image format");
  // counts and histogram bins are 32-bit: a pixel count must fit in 31 bits
  if ((uint64_t)im->w * im->h >= ((uint64_t)1 << 31))
    return set_error(c, HVX_ERROR_INVALID_DIMENSION, "global operators take images of fewer than 2^31 pixels");
  hvx_status s = ensure_device(c);
  if (s) return s;
  gi->base = (const uint8_t*)im->ptr;
  gi->pitch = (int64_t)im->pitch;
  gi->w = (int32_t)im->w;
  gi->h = (int32_t)im->h;
  gi->bpp = df_bytes(im->df);
  return HVX_SUCCESS;
}

static hvx_status launched(hvx_context ctx, hipError_t e) {
  if (e == hipSuccess) return HVX_SUCCESS;
  return set_error(as<Context>(ctx, T_CONTEXT), HVX_ERROR_DEVICE, "kernel launch: %s", hipGetErrorString(e));
}

hvx_status hvx_histogram(hvx_context ctx, hvx_image in, uint32_t num_bins, uint32_t offset, uint32_t range,
                         uint32_t* dev_counts, void* stream) {
  GlobalImg gi;
  hvx_status s = global_input(ctx, in, {DF_U8}, &gi);
  if (s) return s;
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (!dev_counts) return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "null counts buffer");
  if (num_bins < 1 || num_bins > 256 || range < num_bins || offset + (uint64_t)range > 256)
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "need 1 <= num_bins <= range and offset + range <= 256");
  return launched(ctx, launch_histogram(gi, (int)num_bins, (int)offset, (int)range, dev_counts, (hipStream_t)stream));
}

hvx_status hvx_min_max(hvx_context ctx, hvx_image in, int32_t* dev_min_max, void* stream) {
  GlobalImg gi;
  hvx_status s = global_input(ctx, in, {DF_U8, DF_S16}, &gi);
  if (s) return s;
  if (!dev_min_max) return set_error(as<Context>(ctx, T_CONTEXT), HVX_ERROR_INVALID_PARAMETERS, "null result buffer");
  return launched(ctx, launch_min_max(gi, dev_min_max, (hipStream_t)stream));
}

hvx_status hvx_min_max_count(hvx_context ctx, hvx_image in, int32_t* dev_result, void* stream) {
  GlobalImg gi;
  hvx_status s = global_input(ctx, in, {DF_U8, DF_S16}, &gi);
  if (s) return s;
  if (!dev_result || ((uintptr_t)dev_result & 7))
    return set_error(as<Context>(ctx, T_CONTEXT), HVX_ERROR_INVALID_PARAMETERS, "result buffer null or not 8-byte aligned");
  return launched(ctx, launch_min_max_count(gi, dev_result, (hipStream_t)stream));
}

hvx_status hvx_min_max_loc(hvx_context ctx, hvx_image in, int32_t* dev_result, uint32_t* dev_min_locs,
                           uint32_t* dev_max_locs, uint32_t capacity, void* stream) {
  GlobalImg gi;
  hvx_status s = global_input(ctx, in, {DF_U8, DF_S16}, &gi);
  if (s) return s;
  if (!dev_result || ((uintptr_t)dev_result & 7) || (capacity && (!dev_min_locs || !dev_max_locs)))
    return set_error(as<Context>(ctx, T_CONTEXT), HVX_ERROR_INVALID_PARAMETERS,
                     "null result or location buffer, or a result not 8-byte aligned");
  return launched(ctx, launch_min_max_loc(gi, dev_result, dev_min_locs, dev_max_locs, capacity, (hipStream_t)stream));
}

hvx_status hvx_equalize_hist(hvx_context ctx, hvx_image in, hvx_image out, void* dev_workspace, void* stream) {
  GlobalImg gi, go;
  hvx_status s = global_input(ctx, in, {DF_U8}, &gi);
  if (s) return s;
  s = global_input(ctx, out, {DF_U8}, &go);
  if (s) return s;
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (go.w != gi.w || go.h != gi.h) return set_error(c, HVX_ERROR_INVALID_DIMENSION, "output size differs from input");
  if (!dev_workspace || ((uintptr_t)dev_workspace & 3))
    return set_error(c, HVX_ERROR_INVALID_PARAMETERS, "workspace null or not 4-byte aligned");
  return launched(ctx, launch_equalize_hist(gi, (uint8_t*)go.base, go.pitch, dev_workspace, (hipStream_t)stream));
}

hvx_status hvx_equalize_hist_noalloc(hvx_context ctx, hvx_image in, hvx_image out, void* stream) {
  GlobalImg gi, go;
  hvx_status s = global_input(ctx, in, {DF_U8}, &gi);
  if (s) return s;
  s = global_input(ctx, out, {DF_U8}, &go);
  if (s) return s;
  Context* c = as<Context>(ctx, T_CONTEXT);
  if (go.w != gi.w || go.h != gi.h) return set_error(c, HVX_ERROR_INVALID_DIMENSION, "output size differs from input");
  // global_input made the context's device current
  void* ws = nullptr;
  const hipError_t e = equalize_scratch(c->device, &ws);
  if (e != hipSuccess)
    return set_error(c, HVX_ERROR_DEVICE, "device address of the fixed workspace: %s", hipGetErrorString(e));
  return launched(ctx, launch_equalize_hist(gi, (uint8_t*)go.base, go.pitch, ws, (hipStream_t)stream));
}

hvx_status hvx_mean_std_dev(hvx_context ctx, hvx_image in, void* dev_result, void* stream) {
  GlobalImg gi;
  hvx_status s = global_input(ctx, in, {DF_U8}, &gi);
  if (s) return s;
  if (!dev_result || ((uintptr_t)dev_result & 7))
    return set_error(as<Context>(ctx, T_CONTEXT), HVX_ERROR_INVALID_PARAMETERS, "result buffer null or not 8-byte aligned");
  return launched(ctx, launch_mean_std_dev(gi, dev_result, (hipStream_t)stream));
}

hvx_status hvx_custom_local_node(hvx_graph g, const char* expr, hvx_image in, int out_format, hvx_image out,
                                 hvx_node* no) {
  Graph* gg = as<Graph>(g, T_GRAPH);
  if (!gg) return HVX_ERROR_INVALID_REFERENCE;
  if (out_format != HVX_DF_U8 && out_format != HVX_DF_S16 && out_format != HVX_DF_F32)
    return set_error(gg->ctx, HVX_ERROR_INVALID_FORMAT, "output format must be U8, S16 or F32");
  ExprProg prog;
  std::string why = parse_expr(expr, &prog);
  if (!why.empty()) return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "expression: %s", why.c_str());
  if (prog.max_input > 0)
    return set_error(gg->ctx, HVX_ERROR_INVALID_PARAMETERS, "a user local kernel has one input, a");
  Node* n = nullptr;
  hvx_status s = add_node(g, NK_CUSTOM_LOCAL, {in}, {out}, 1, no, &n);
  if (s) return s;
  n->expr = std::move(prog);
  n->out_df = out_format;
  return HVX_SUCCESS;
}

hvx_status hvx_node_set_border(hvx_node node, int border, uint32_t constant_value) {
  Node* n = as<Node>(node, T_NODE);
  if (!n) return HVX_ERROR_INVALID_REFERENCE;
  if (border != B_UNDEFINED && border != B_CONSTANT && border != B_REPLICATE && border != B_MIRROR &&
      border != B_REPEAT)
    return set_error(n->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown border mode %d", border);
  n->border = border;
  n->bconst = constant_value;
  invalidate(n->g);
  return HVX_SUCCESS;
}

hvx_status hvx_graph_set_option(hvx_graph graph, int option, int64_t value) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  switch (option) {
    case HVX_OPT_FUSION: g->opt_fusion = value != 0; break;
    case HVX_OPT_DCE: g->opt_dce = value != 0; break;
    case HVX_OPT_TILE:
      if (value < 0 || value > 65536) return set_error(g->ctx, HVX_ERROR_INVALID_PARAMETERS, "bad tile rows");
      g->opt_tile = (int)value;
      break;
    case HVX_OPT_SPECIALIZE: g->opt_specialize = value != 0; break;
    case HVX_OPT_XCD_REMAP: g->opt_xcd = value != 0; break;
    case HVX_OPT_CODEGEN: g->opt_codegen = value != 0; break;
    default: return set_error(g->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown option %d", option);
  }
  invalidate(g);
  return HVX_SUCCESS;
}

hvx_status hvx_graph_verify(hvx_graph graph) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  std::lock_guard<std::recursive_mutex> l(g->ctx->mu);
  invalidate(g);
  return verify_graph(g);
}

hvx_status hvx_graph_schedule(hvx_graph graph, void* stream) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  if (!g->verified) {
    hvx_status s = verify_graph(g);
    if (s) return s;
  }
  return schedule_graph(g, stream);
}

hvx_status hvx_graph_wait(hvx_graph graph) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  if (!g->scheduled) return HVX_SUCCESS;
  hipError_t e = hipStreamSynchronize((hipStream_t)g->last_stream);
  if (e != hipSuccess) return set_error(g->ctx, HVX_ERROR_DEVICE, "stream sync: %s", hipGetErrorString(e));
  g->scheduled = false;
  return HVX_SUCCESS;
}

hvx_status hvx_graph_process(hvx_graph graph) {
  hvx_status s = hvx_graph_schedule(graph, nullptr);
  if (s) return s;
  return hvx_graph_wait(graph);
}

hvx_status hvx_graph_query(hvx_graph graph, int attr, int64_t* out) {
  Graph* g = as<Graph>(graph, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  if (!out) return set_error(g->ctx, HVX_ERROR_INVALID_PARAMETERS, "null output");
  if (attr == HVX_QUERY_NUM_NODES) {
    *out = (int64_t)g->nodes.size();
    return HVX_SUCCESS;
  }
  if (!g->verified || !g->plan) return set_error(g->ctx, HVX_ERROR_NOT_VERIFIED, "graph is not verified");
  const Plan& p = *g->plan;
  switch (attr) {
    case HVX_QUERY_NUM_OPS: *out = p.num_ops; break;
    case HVX_QUERY_NUM_LIVE_OPS: *out = p.num_live; break;
    case HVX_QUERY_NUM_KERNELS: *out = (int64_t)p.groups.size(); break;
    case HVX_QUERY_ALG_BYTES: *out = p.alg_bytes; break;
    case HVX_QUERY_HBM_BYTES: *out = p.hbm_bytes; break;
    case HVX_QUERY_KERNEL_KIND: *out = p.groups.empty() ? -1 : p.groups[0].kind; break;
    case HVX_QUERY_SCRATCH_BYTES: *out = p.scratch_bytes; break;
    case HVX_QUERY_OP_LIVE_MASK: {
      int64_t m = 0;
      for (size_t i = 0; i < p.ops.size() && i < 63; ++i)
        if (p.ops[i].live) m |= (int64_t)1 << i;
      *out = m;
      break;
    }
    case HVX_QUERY_ROWS_PER_ITEM:
      *out = (p.groups.empty() || !is_strip_kind(p.groups[0].kind)) ? 0 : rows_for(g, p.groups[0]);
      break;
    case HVX_QUERY_NUM_GENERATED: *out = p.num_generated; break;
    case HVX_QUERY_PLAN_CUTS: *out = (int64_t)p.cuts.size(); break;
    case HVX_QUERY_GEN_TILE:
      *out = p.tiles.empty() ? 0 : ((int64_t)p.tiles[0][1] << 16 | p.tiles[0][2]);
      break;
    default: return set_error(g->ctx, HVX_ERROR_INVALID_PARAMETERS, "unknown query %d", attr);
  }
  return HVX_SUCCESS;
}

// ---- release ----------------------------------------------------------------

hvx_status hvx_release_graph(hvx_graph* pg) {
  if (!pg) return HVX_ERROR_INVALID_PARAMETERS;
  Graph* g = as<Graph>(*pg, T_GRAPH);
  if (!g) return HVX_ERROR_INVALID_REFERENCE;
  if (g->scheduled) (void)hipStreamSynchronize((hipStream_t)g->last_stream);
  remove_child(g->ctx, g);
  destroy_graph(g);
  *pg = nullptr;
  return HVX_SUCCESS;
}

hvx_status hvx_release_image(hvx_image* pi) {
  if (!pi) return HVX_ERROR_INVALID_PARAMETERS;
  Image* im = as<Image>(*pi, T_IMAGE);
  if (!im) return HVX_ERROR_INVALID_REFERENCE;
  // Images still referenced by a node of a live graph stay allocated until
  // that graph or the context is released; the handle becomes invalid now.
  Context* c = im->ctx;
  bool used = false;
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    for (Object* o : c->children) {
      if (o->type != T_GRAPH) continue;
      for (Node* n : ((Graph*)o)->nodes) {
        for (Image* x : n->in) used |= x == im;
        for (Image* x : n->out) used |= x == im;
      }
    }
  }
  if (used) {
    // still wired into a graph: the handle is retired now, the object lives
    // on with its graph (virtual) or its context (non-virtual)
    registry_remove(im);
    *pi = nullptr;
    return HVX_SUCCESS;
  }
  if (im->is_virtual) {
    auto& v = im->vgraph->virt;
    v.erase(std::remove(v.begin(), v.end(), im), v.end());
    destroy_image(im);
    *pi = nullptr;
    return HVX_SUCCESS;
  }
  remove_child(c, im);
  destroy_image(im);
  *pi = nullptr;
  return HVX_SUCCESS;
}

hvx_status hvx_release_node(hvx_node* pn) {
  if (!pn) return HVX_ERROR_INVALID_PARAMETERS;
  Node* n = as<Node>(*pn, T_NODE);
  if (!n) return HVX_ERROR_INVALID_REFERENCE;
  // As in OpenVX, releasing a node's handle does not remove the node from its
  // graph; the node is freed with the graph.
  registry_remove(n);
  *pn = nullptr;
  return HVX_SUCCESS;
}

hvx_status hvx_release_convolution(hvx_convolution* pc) {
  if (!pc) return HVX_ERROR_INVALID_PARAMETERS;
  Conv* cv = as<Conv>(*pc, T_CONV);
  if (!cv) return HVX_ERROR_INVALID_REFERENCE;
  Context* c = cv->ctx;
  bool used = false;
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    for (Object* o : c->children)
      if (o->type == T_GRAPH)
        for (Node* n : ((Graph*)o)->nodes) used |= n->conv == cv;
  }
  registry_remove(cv);
  if (!used) {
    remove_child(c, cv);
    delete cv;
  }
  *pc = nullptr;
  return HVX_SUCCESS;
}

hvx_status hvx_release_buffer(hvx_buffer* pb) {
  if (!pb) return HVX_ERROR_INVALID_PARAMETERS;
  Image* b = as<Image>(*pb, T_BUFFER);
  if (!b) return HVX_ERROR_INVALID_REFERENCE;
  Context* c = b->ctx;
  bool used = false;
  {
    std::lock_guard<std::recursive_mutex> l(c->mu);
    for (Object* o : c->children)
      if (o->type == T_GRAPH)
        for (Node* n : ((Graph*)o)->nodes)
          for (Image* x : n->out) used |= x == b;
  }
  registry_remove(b);
  if (!used) {
    remove_child(c, b);
    delete b;
  }
  *pb = nullptr;
  return HVX_SUCCESS;
}

}  // extern "C"
