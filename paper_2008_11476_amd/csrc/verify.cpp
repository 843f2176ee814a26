// Graph verification and planning (host only, no device work).
//
// Order of the passes (Sections 3.1 and 5.2):
//   1. parameter presence, ownership of virtual images, single writer per
//      image, bipartite node/data structure, no cycles;
//   2. virtual-image inference and per-node format and size checks;
//   3. lowering of every function node to point/local operators (Section 4,
//      Table 2; Sobel becomes two local operators, Section 5.2.2);
//   4. elimination of dead computations (Section 5.2.2, Algorithm 1);
//   5. transfer reduction and fusion: live operators of one connected
//      component form one kernel whose virtual intermediates never reach
//      device memory (Sections 5.2.1 and 6.3);
//   6. kernel choice (hand-fused kernel for a recognised subgraph, else the
//      generic tile interpreter) and its program / launch shape.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <set>

#include "codegen.h"
#include "hvx_internal.h"

namespace hvx {

static int op_radius(const LOp& o, int* rx, int* ry) {
  int r = 0;
  switch (o.kind) {
    case OP_GAUSS3:
    case OP_BOX3:
    case OP_DILATE3:
    case OP_ERODE3:
    case OP_MEDIAN3:
    case OP_SOBEL_X:
    case OP_SOBEL_Y: r = 1; break;
    case OP_GAUSS5:
    case OP_BOX5F: r = 2; break;
    case OP_NONMAX: r = o.policy / 2; break;  // the window size
    case OP_EXPR_LOCAL:
      *rx = o.expr->rx;
      *ry = o.expr->ry;
      return std::max(*rx, *ry);
    case OP_CONVOLVE:
    case OP_NONLINEAR:
      *rx = (int)o.conv->cols / 2;
      *ry = (int)o.conv->rows / 2;
      return std::max(*rx, *ry);
    default: r = 0;
  }
  *rx = *ry = r;
  return r;
}

static bool is_int_df(int df) { return df == DF_U8 || df == DF_S16 || df == DF_S32; }

// ---- 1 + 2: structure checks and inference ----------------------------------

struct Builder {
  Graph* g;
  Plan* p;
  std::map<Image*, int> vid;

  int value_of(Image* im) {
    auto it = vid.find(im);
    if (it != vid.end()) return it->second;
    Value v;
    v.img = im;
    v.is_virtual = im->is_virtual;
    v.df = im->df;
    v.w = im->w;
    v.h = im->h;
    p->vals.push_back(v);
    int id = (int)p->vals.size() - 1;
    vid[im] = id;
    return id;
  }
};

static hvx_status err(Graph* g, hvx_status s, const char* fmt, const char* a = "", int b = 0) {
  return set_error(g->ctx, s, fmt, a, b);
}

static const char* node_name(int kind) {
  switch (kind) {
    case NK_CHANNEL_EXTRACT: return "ChannelExtract";
    case NK_GAUSS3: return "Gaussian3x3";
    case NK_GAUSS5: return "Gaussian5x5";
    case NK_BOX3: return "Box3x3";
    case NK_DILATE3: return "Dilate3x3";
    case NK_ERODE3: return "Erode3x3";
    case NK_MEDIAN3: return "Median3x3";
    case NK_NONLINEAR: return "NonLinearFilter";
    case NK_NONMAX: return "NonMaxSuppression";
    case NK_CUSTOM_POINT: return "user point kernel";
    case NK_CUSTOM_LOCAL: return "user local kernel";
    case NK_BOX5F: return "Box5x5F32";
    case NK_SOBEL3: return "Sobel3x3";
    case NK_MAGNITUDE: return "Magnitude";
    case NK_PHASE: return "Phase";
    case NK_ADD: return "Add";
    case NK_MULF: return "MultiplyF32";
    case NK_HARRIS: return "HarrisResponse";
    case NK_THRESHOLD: return "Threshold";
    case NK_CONVOLVE: return "Convolve";
    case NK_HISTOGRAM: return "Histogram";
    case NK_MINMAX: return "MinMax";
    case NK_MINMAXLOC: return "MinMaxLoc";
    case NK_MEANSTD: return "MeanStdDev";
    case NK_EQHIST: return "EqualizeHist";
    default: return "?";
  }
}

// Resolve/check one output value against the format/size the node produces.
static hvx_status bind_output(Graph* g, Plan& p, int v, int df, uint32_t w, uint32_t h, const char* nn) {
  Value& val = p.vals[v];
  if (val.is_virtual) {
    if (val.img->df != DF_VIRT && val.img->df != df)
      return err(g, HVX_ERROR_INVALID_FORMAT, "%s: virtual output declared with a different format", nn);
    if (val.img->w != 0 && (val.img->w != w || val.img->h != h))
      return err(g, HVX_ERROR_INVALID_DIMENSION, "%s: virtual output declared with a different size", nn);
    val.df = df;
    val.w = w;
    val.h = h;
    return HVX_SUCCESS;
  }
  if (val.df != df) return err(g, HVX_ERROR_INVALID_FORMAT, "%s: output image has the wrong format", nn);
  if (val.w != w || val.h != h) return err(g, HVX_ERROR_INVALID_DIMENSION, "%s: output size differs from input", nn);
  return HVX_SUCCESS;
}

// A global operator's result buffer: must be one and hold `need` bytes.
static hvx_status bind_buffer(Graph* g, Plan& p, int v, int64_t need, const char* nn) {
  const Value& val = p.vals[v];
  if (val.df != DF_BUF) return err(g, HVX_ERROR_INVALID_FORMAT, "%s writes its result to a buffer", nn);
  if ((int64_t)val.w < need)
    return err(g, HVX_ERROR_INVALID_DIMENSION, "%s: result buffer too small (needs %d bytes)", nn, (int)need);
  return HVX_SUCCESS;
}

// ---- 6: kernel choice --------------------------------------------------------

static int producer_in(const Plan& p, int v, const std::set<int>& ops) {
  int pr = p.vals[v].producer;
  return (pr >= 0 && ops.count(pr)) ? pr : -1;
}

// Gaussian3x3 -> SobelX, SobelY -> Magnitude -> Threshold (+ Phase(gx, gy)).
// The hand-fused kernels implement the UNDEFINED, CONSTANT and REPLICATE
// borders; a group with a MIRROR or REPEAT border runs on the generic kernels.
static bool fast_borders(const Plan& p, const Group& gr) {
  for (int o : gr.ops)
    if (p.ops[o].border == B_MIRROR || p.ops[o].border == B_REPEAT) return false;
  return true;
}

// A local operator with the REPEAT border reads its input at the far side of
// the image.  A tile holds an intermediate only around itself, so such an
// operator must read a value that is in memory: a group where it reads one
// computed inside the group runs node by node.
static bool repeat_reads_intermediate(const Plan& p, const Group& gr) {
  std::set<int> ops(gr.ops.begin(), gr.ops.end());
  for (int o : gr.ops) {
    const LOp& op = p.ops[o];
    int rx, ry;
    if (op.border != B_REPEAT || op_radius(op, &rx, &ry) == 0) continue;
    for (int k = 0; k < op.nin; ++k)
      if (producer_in(p, op.in[k], ops) >= 0) return true;
  }
  return false;
}

static bool match_edge(const Plan& p, const Group& gr, int* in_v, int* out_v, int* ph_v) {
  if (gr.ops.size() != 5 && gr.ops.size() != 6) return false;
  std::set<int> ops(gr.ops.begin(), gr.ops.end());
  int thr = -1, phs = -1;
  for (int o : gr.ops) {
    if (p.ops[o].kind == OP_THRESHOLD) thr = o;
    if (p.ops[o].kind == OP_PHASE) phs = o;
  }
  if (thr < 0 || (gr.ops.size() == 6) != (phs >= 0)) return false;
  const LOp& t = p.ops[thr];
  if (p.vals[t.in[0]].df != DF_S16) return false;
  int mag = producer_in(p, t.in[0], ops);
  if (mag < 0 || p.ops[mag].kind != OP_MAGNITUDE) return false;
  int a = producer_in(p, p.ops[mag].in[0], ops), b = producer_in(p, p.ops[mag].in[1], ops);
  if (a < 0 || b < 0 || a == b) return false;
  int sx = p.ops[a].kind == OP_SOBEL_X ? a : b, sy = p.ops[a].kind == OP_SOBEL_X ? b : a;
  if (p.ops[sx].kind != OP_SOBEL_X || p.ops[sy].kind != OP_SOBEL_Y) return false;
  if (p.ops[sx].in[0] != p.ops[sy].in[0]) return false;
  if (p.ops[sx].border != p.ops[sy].border || p.ops[sx].bconst != p.ops[sy].bconst) return false;
  int ga = producer_in(p, p.ops[sx].in[0], ops);
  if (ga < 0 || p.ops[ga].kind != OP_GAUSS3) return false;
  if (producer_in(p, p.ops[ga].in[0], ops) >= 0) return false;
  if (phs >= 0) {
    if (p.ops[phs].in[0] != p.ops[sx].out || p.ops[phs].in[1] != p.ops[sy].out) return false;
  }
  // intermediates must stay inside the group (virtual and not read outside)
  for (int v : {p.ops[ga].out, p.ops[sx].out, p.ops[sy].out, p.ops[mag].out}) {
    if (!p.vals[v].is_virtual) return false;
    for (int c : p.vals[v].consumers)
      if (!ops.count(c)) return false;
  }
  *in_v = p.ops[ga].in[0];
  *out_v = t.out;
  *ph_v = phs >= 0 ? p.ops[phs].out : -1;
  return p.vals[*in_v].df == DF_U8 && !p.vals[*in_v].is_virtual && !p.vals[*out_v].is_virtual &&
         (*ph_v < 0 || !p.vals[*ph_v].is_virtual);
}

// SobelX, SobelY -> gx*gx, gy*gy, gx*gy -> Box5x5 (x3) -> response -> Threshold.
static bool match_corner(const Plan& p, const Group& gr, int* in_v, int* out_v) {
  if (gr.ops.size() != 10) return false;
  std::set<int> ops(gr.ops.begin(), gr.ops.end());
  int thr = -1;
  for (int o : gr.ops)
    if (p.ops[o].kind == OP_THRESHOLD) thr = o;
  if (thr < 0) return false;
  const LOp& t = p.ops[thr];
  int hr = producer_in(p, t.in[0], ops);
  if (hr < 0 || p.ops[hr].kind != OP_HARRIS) return false;
  int sx = -1, sy = -1;
  int box[3], mul[3];
  for (int i = 0; i < 3; ++i) {
    box[i] = producer_in(p, p.ops[hr].in[i], ops);
    if (box[i] < 0 || p.ops[box[i]].kind != OP_BOX5F) return false;
    mul[i] = producer_in(p, p.ops[box[i]].in[0], ops);
    if (mul[i] < 0 || p.ops[mul[i]].kind != OP_MULF) return false;
  }
  for (int i = 1; i < 3; ++i)
    if (p.ops[box[i]].border != p.ops[box[0]].border || p.ops[box[i]].bconst != p.ops[box[0]].bconst) return false;
  // the fast kernel sums exactly in int32: 25 * constant must stay in range
  if (p.ops[box[0]].border == B_CONSTANT && p.ops[box[0]].bconst > 1040400u) return false;
  // identify gradients
  for (int o : gr.ops) {
    if (p.ops[o].kind == OP_SOBEL_X) sx = o;
    if (p.ops[o].kind == OP_SOBEL_Y) sy = o;
  }
  if (sx < 0 || sy < 0 || p.ops[sx].in[0] != p.ops[sy].in[0]) return false;
  if (p.ops[sx].border != p.ops[sy].border || p.ops[sx].bconst != p.ops[sy].bconst) return false;
  int gx = p.ops[sx].out, gy = p.ops[sy].out;
  auto is_prod = [&](int m, int a, int b) {
    return (p.ops[m].in[0] == a && p.ops[m].in[1] == b) || (p.ops[m].in[0] == b && p.ops[m].in[1] == a);
  };
  bool ok01 = (is_prod(mul[0], gx, gx) && is_prod(mul[1], gy, gy)) || (is_prod(mul[0], gy, gy) && is_prod(mul[1], gx, gx));
  if (!ok01 || !is_prod(mul[2], gx, gy)) return false;
  if (producer_in(p, p.ops[sx].in[0], ops) >= 0) return false;
  for (int o : gr.ops) {
    if (o == thr) continue;
    int v = p.ops[o].out;
    if (!p.vals[v].is_virtual) return false;
    for (int c : p.vals[v].consumers)
      if (!ops.count(c)) return false;
  }
  *in_v = p.ops[sx].in[0];
  *out_v = t.out;
  return p.vals[*in_v].df == DF_U8 && !p.vals[*in_v].is_virtual && !p.vals[*out_v].is_virtual;
}

// Gaussian5x5 of a U8 image, or of the luma of a UYVY frame.
static bool match_gauss5(const Plan& p, const Group& gr, int* in_v, int* out_v) {
  if (gr.ops.size() == 1) {
    const LOp& o = p.ops[gr.ops[0]];
    if (o.kind != OP_GAUSS5) return false;
    *in_v = o.in[0];
    *out_v = o.out;
    return !p.vals[*in_v].is_virtual && !p.vals[*out_v].is_virtual;
  }
  if (gr.ops.size() == 2) {
    const LOp& a = p.ops[gr.ops[0]];
    const LOp& b = p.ops[gr.ops[1]];
    if (a.kind != OP_CHANNEL_Y || b.kind != OP_GAUSS5 || b.in[0] != a.out) return false;
    if (!p.vals[a.out].is_virtual || p.vals[a.out].consumers.size() != 1) return false;
    *in_v = a.in[0];
    *out_v = b.out;
    return !p.vals[*in_v].is_virtual && !p.vals[*out_v].is_virtual;
  }
  return false;
}

// ---- generic program ------------------------------------------------------------

static bool build_generic(Graph* g, Plan& p, Group& gr, std::string* why) {
  GProg& P = gr.prog;
  memset(&P, 0, sizeof P);
  std::set<int> ops(gr.ops.begin(), gr.ops.end());
  std::vector<int> vals;  // group-local value list
  std::map<int, int> loc;
  auto local = [&](int v) {
    auto it = loc.find(v);
    if (it != loc.end()) return it->second;
    loc[v] = (int)vals.size();
    vals.push_back(v);
    return (int)vals.size() - 1;
  };
  for (int v : gr.inputs) local(v);
  for (int o : gr.ops) local(p.ops[o].out);
  if ((int)vals.size() > kMaxGVals || (int)gr.ops.size() > kMaxGOps) {
    *why = "too many values or operators for one kernel";
    return false;
  }
  int nio = (int)(gr.inputs.size() + gr.outputs.size());
  if (nio > kMaxIO) {
    *why = "too many inputs/outputs for one kernel";
    return false;
  }
  std::set<int> outset(gr.outputs.begin(), gr.outputs.end());
  // global operators reduced over the tiles: at most kMaxRed, one of them a
  // histogram (its counters take LDS next to the tiles)
  int nred = 0, nhist = 0;
  for (int o : gr.ops) {
    const int k = p.ops[o].kind;
    if (k == OP_MMLOCS) {
      *why = "the location pass runs alone";
      return false;
    }
    nred += is_reduce_op(k) ? 1 : 0;
    nhist += (k == OP_HISTOGRAM || k == OP_EQHIST) ? 1 : 0;
  }
  if (nred > kMaxRed || nhist > 1) {
    *why = "too many global operators for one kernel";
    return false;
  }
  // halo extents, consumers first
  std::vector<int> ext(vals.size(), 0);
  std::vector<int> read_in_group(vals.size(), 0);
  for (int i = (int)gr.ops.size() - 1; i >= 0; --i) {
    const LOp& o = p.ops[gr.ops[i]];
    int rx, ry;
    int r = op_radius(o, &rx, &ry);
    int eo = ext[loc[o.out]];
    for (int k = 0; k < o.nin; ++k) {
      int li = loc[o.in[k]];
      ext[li] = std::max(ext[li], eo + r);
      read_in_group[li] = 1;
    }
  }
  gr.footprint = 0;
  for (size_t i = 0; i < vals.size(); ++i) gr.footprint = std::max(gr.footprint, ext[i]);
  // liveness of on-chip values: [def, last use] in op order; inputs defined at -1
  std::vector<int> def(vals.size(), -1), last(vals.size(), -2);
  for (size_t i = 0; i < gr.ops.size(); ++i) {
    const LOp& o = p.ops[gr.ops[i]];
    def[loc[o.out]] = (int)i;
    for (int k = 0; k < o.nin; ++k) last[loc[o.in[k]]] = std::max(last[loc[o.in[k]]], (int)i);
  }
  // choose the tile: shrink until the live set fits the LDS budget
  const int budget_words = 48 * 1024 / 4 - (nhist ? kHistWords : 0);
  static const int shapes[][2] = {{64, 16}, {64, 8}, {32, 8}, {32, 4}, {16, 4}};
  for (auto& sh : shapes) {
    int tw = sh[0], th = sh[1];
    std::vector<int> off(vals.size(), -1), size(vals.size(), 0);
    // first-fit interval allocation, values in definition order
    int top = 0;
    std::vector<int> order(vals.size());
    for (size_t i = 0; i < vals.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return def[a] < def[b]; });
    std::vector<std::array<int, 3>> blocks;  // offset, size, last use
    for (int li : order) {
      if (!read_in_group[li] || p.vals[vals[li]].df == DF_BUF) continue;  // buffers stay in memory
      int e = ext[li];
      int sz = (tw + 2 * e) * (th + 2 * e);
      size[li] = sz;
      // blocks freed before this value's definition can be reused
      std::vector<std::array<int, 3>> live;
      for (auto& b : blocks)
        if (b[2] >= def[li]) live.push_back(b);
      std::sort(live.begin(), live.end());
      int pos = 0;
      for (auto& b : live) {
        if (pos + sz <= b[0]) break;
        pos = std::max(pos, b[0] + b[1]);
      }
      off[li] = pos;
      top = std::max(top, pos + sz);
      blocks.push_back({pos, sz, last[li]});
    }
    if (top <= budget_words) {
      P.tw = tw;
      P.th = th;
      P.lds_words = top;
      for (size_t i = 0; i < vals.size(); ++i) P.vals[i].lds = off[i];
      break;
    }
  }
  if (P.tw == 0) {
    *why = "live intermediates exceed the LDS budget";
    return false;
  }
  P.nvals = (int)vals.size();
  P.nops = (int)gr.ops.size();
  P.nred = nred;
  gr.gvals = vals;
  P.w = (int)gr.w;
  P.h = (int)gr.h;
  P.tiles_x = (P.w + P.tw - 1) / P.tw;
  P.tiles_y = (P.h + P.th - 1) / P.th;
  int io = 0;
  for (size_t i = 0; i < vals.size(); ++i) {
    int v = vals[i];
    GVal& gv = P.vals[i];
    gv.df = p.vals[v].df;
    gv.ext = ext[i];
    gv.input = std::find(gr.inputs.begin(), gr.inputs.end(), v) != gr.inputs.end();
    gv.store = outset.count(v) ? 1 : 0;
    gv.io = (gv.input || gv.store) ? io++ : -1;
    gv.wrap = 0;
    for (int o : gr.ops) {
      const LOp& op = p.ops[o];
      int rx, ry;
      if (gv.input && op.border == B_REPEAT && op_radius(op, &rx, &ry) > 0)
        for (int k = 0; k < op.nin; ++k) gv.wrap |= op.in[k] == v;
    }
  }
  for (size_t i = 0; i < gr.ops.size(); ++i) {
    const LOp& o = p.ops[gr.ops[i]];
    GOp& q = P.ops[i];
    q.kind = o.kind;
    q.out = loc[o.out];
    for (int k = 0; k < 3; ++k) q.in[k] = k < o.nin ? loc[o.in[k]] : -1;
    q.border = o.border;
    int in_df = o.nin ? p.vals[o.in[0]].df : DF_U8;
    // the constant is read as the input's element type
    if (in_df == DF_U8) q.cint = (int)std::min<uint32_t>(o.bconst, 255);
    else if (in_df == DF_S16) q.cint = (int)(int16_t)(uint16_t)o.bconst;
    else q.cint = (int)o.bconst;
    q.cf = (float)o.bconst;
    op_radius(o, &q.rx, &q.ry);
    switch (o.kind) {
      case OP_THRESHOLD: {
        q.p0 = o.tv;
        q.p1 = o.fv;
        // integer inputs: in > t  <=>  in >= floor(t) + 1
        double u = floor(o.dval) + 1.0;
        q.p2 = u < -2147483647.0 ? -2147483647 : (u > 2147483647.0 ? 2147483647 : (int)u);
        // float inputs: in > t  <=>  in > (largest float not above t)
        float f = (float)o.dval;
        if ((double)f > o.dval) f = nextafterf(f, -INFINITY);
        q.pf = f;
        break;
      }
      case OP_ADD: q.p0 = o.policy; break;
      case OP_HARRIS: q.pf = o.k; break;
      case OP_HISTOGRAM:
        q.p0 = (int)o.gp[0];
        q.p1 = (int)o.gp[1];
        q.p2 = (int)o.gp[2];
        break;
      case OP_EQHIST:
        q.p0 = 256;
        q.p1 = 0;
        q.p2 = 256;
        break;
      case OP_NONMAX: q.p0 = o.policy / 2; break;
      case OP_EXPR:
      case OP_EXPR_LOCAL: {
        const ExprProg& e = *o.expr;
        q.p0 = (int)e.code.size();
        q.p1 = P.vals[q.out].df == DF_F32 ? 1 : 0;
        q.p2 = 0;
        for (int k = 0; k < o.nin; ++k) q.p2 |= (P.vals[q.in[k]].df == DF_F32 ? 1 : 0) << k;
        for (size_t k = 0; k < e.code.size(); ++k) q.code[k] = e.code[k];
        for (size_t k = 0; k < e.consts.size(); ++k) {
          if (q.p1) {
            const float f = (float)e.consts[k];
            memcpy(&q.kc[k], &f, 4);
          } else {
            q.kc[k] = (int32_t)e.consts[k];
          }
        }
        break;
      }
      case OP_NONLINEAR:
        q.p0 = (int)o.conv->cols;
        q.p1 = (int)o.conv->rows;
        q.p2 = o.policy;
        for (size_t k = 0; k < o.conv->coeffs.size(); ++k) q.mask[k] = o.conv->coeffs[k];
        break;
      case OP_CONVOLVE: {
        q.p0 = (int)o.conv->cols;
        q.p1 = (int)o.conv->rows;
        int sh = 0;
        while ((1u << sh) < o.conv->scale) ++sh;
        q.p2 = sh;
        for (size_t k = 0; k < o.conv->coeffs.size(); ++k) q.mask[k] = o.conv->coeffs[k];
        break;
      }
      default: break;
    }
  }
  (void)g;
  return true;
}

// threshold of gx^2+gy^2 equivalent to round(sqrt) > t (see EdgeDesc)
int32_t edge_threshold_not(double t) {
  double u = floor(t) + 1.0;
  int64_t T;
  if (u <= 0) T = -1;
  else if (u > 32767) T = 2147483647;
  else T = (int64_t)u * ((int64_t)u - 1);
  return ~(int32_t)T;
}

// ---- verify ---------------------------------------------------------------------

hvx_status verify_graph(Graph* g) {
  g->verified = false;
  g->plan.reset();
  std::unique_ptr<Plan> pp(new Plan());
  Plan& p = *pp;
  Builder B{g, &p, {}};
  const int N = (int)g->nodes.size();
  p.num_nodes = N;
  if (N == 0) return err(g, HVX_ERROR_INVALID_GRAPH, "graph has no nodes");

  // node -> value ids
  std::vector<std::vector<int>> nin(N), nout(N);
  for (int i = 0; i < N; ++i) {
    Node* n = g->nodes[i];
    for (Image* im : n->in) {
      if (!registry_check(im, T_IMAGE) && !(im && im->type == T_IMAGE))
        return err(g, HVX_ERROR_INVALID_REFERENCE, "%s: input image was released", node_name(n->kind));
      if (im->is_virtual && im->vgraph != g)
        return err(g, HVX_ERROR_INVALID_GRAPH, "%s: virtual image of another graph", node_name(n->kind));
      nin[i].push_back(B.value_of(im));
    }
    for (Image* im : n->out) {
      if (!im) {
        nout[i].push_back(-1);
        continue;
      }
      if (im->is_virtual && im->vgraph != g)
        return err(g, HVX_ERROR_INVALID_GRAPH, "%s: virtual image of another graph", node_name(n->kind));
      nout[i].push_back(B.value_of(im));
    }
  }
  // single writer per image; a node may not read what it writes
  std::vector<int> writer(p.vals.size(), -1);
  for (int i = 0; i < N; ++i)
    for (int v : nout[i]) {
      if (v < 0) continue;
      if (writer[v] >= 0) return err(g, HVX_ERROR_INVALID_GRAPH, "an image has two writers (%s)", node_name(g->nodes[i]->kind));
      writer[v] = i;
      for (int u : nin[i])
        if (u == v) return err(g, HVX_ERROR_INVALID_GRAPH, "%s reads its own output (cycle)", node_name(g->nodes[i]->kind));
    }
  // bipartite check over the edge list: every edge joins a data vertex and a node vertex
  {
    const int V = (int)p.vals.size();  // data vertices 0..V-1, node vertices V..V+N-1
    for (int i = 0; i < N; ++i) {
      for (int v : nin[i])
        if (!(v >= 0 && v < V)) return err(g, HVX_ERROR_INVALID_GRAPH, "edge between two node vertices");
      for (int v : nout[i])
        if (v >= V) return err(g, HVX_ERROR_INVALID_GRAPH, "edge between two node vertices");
    }
  }
  // cycle check and topological order of nodes (Kahn)
  std::vector<int> indeg(N, 0);
  std::vector<std::vector<int>> succ(N);
  for (int i = 0; i < N; ++i)
    for (int v : nin[i])
      if (writer[v] >= 0) {
        succ[writer[v]].push_back(i);
        ++indeg[i];
      }
  std::vector<int> order;
  for (int i = 0; i < N; ++i)
    if (!indeg[i]) order.push_back(i);
  for (size_t k = 0; k < order.size(); ++k)
    for (int s : succ[order[k]])
      if (--indeg[s] == 0) order.push_back(s);
  if ((int)order.size() != N) return err(g, HVX_ERROR_INVALID_GRAPH, "graph has a cycle");

  // inference and checks in dependency order
  for (int i : order) {
    Node* n = g->nodes[i];
    const char* nn = node_name(n->kind);
    for (int v : nin[i]) {
      Value& val = p.vals[v];
      if (val.is_virtual && writer[v] < 0) return err(g, HVX_ERROR_INVALID_GRAPH, "%s reads a virtual image nobody writes", nn);
      if (val.df == DF_VIRT || val.w == 0)
        return err(g, HVX_ERROR_INVALID_GRAPH, "%s: input format or size unresolved", nn);
    }
    const Value& a = p.vals[nin[i][0]];
    uint32_t w = a.w, h = a.h;
    for (int v : nin[i])
      if (p.vals[v].w != w || p.vals[v].h != h)
        return err(g, HVX_ERROR_INVALID_DIMENSION, "%s: inputs differ in size", nn);
    auto need = [&](int v, std::initializer_list<int> ok) {
      for (int d : ok)
        if (p.vals[v].df == d) return true;
      return false;
    };
    hvx_status s = HVX_SUCCESS;
    switch (n->kind) {
      case NK_CHANNEL_EXTRACT:
        if (!need(nin[i][0], {DF_UYVY})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a UYVY input", nn);
        s = bind_output(g, p, nout[i][0], DF_U8, w, h, nn);
        break;
      case NK_GAUSS3:
      case NK_GAUSS5:
      case NK_BOX3:
      case NK_DILATE3:
      case NK_ERODE3:
      case NK_MEDIAN3:
      case NK_NONLINEAR:
        if (!need(nin[i][0], {DF_U8})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8 input", nn);
        s = bind_output(g, p, nout[i][0], DF_U8, w, h, nn);
        break;
      case NK_CUSTOM_POINT:
      case NK_CUSTOM_LOCAL: {
        // a float kernel (an F32 input or output) has an F32 output; an
        // integer kernel uses no sqrt and only 32-bit integer literals
        bool flt = n->out_df == DF_F32;
        for (int v : nin[i]) {
          if (!need(v, {DF_U8, DF_S16, DF_F32})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs U8/S16/F32 inputs", nn);
          flt |= p.vals[v].df == DF_F32;
        }
        if (flt && n->out_df != DF_F32)
          return err(g, HVX_ERROR_INVALID_FORMAT, "%s: a kernel with an F32 input has an F32 output", nn);
        if (!flt && (n->expr.needs_float || !n->expr.int_literals_ok))
          return err(g, HVX_ERROR_INVALID_FORMAT, "%s: sqrt and non-integer literals need a float kernel", nn);
        s = bind_output(g, p, nout[i][0], n->out_df, w, h, nn);
        break;
      }
      case NK_NONMAX:
        if (!need(nin[i][0], {DF_U8, DF_S16})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8/S16 input", nn);
        s = bind_output(g, p, nout[i][0], p.vals[nin[i][0]].df, w, h, nn);
        break;
      case NK_BOX5F:
        if (!need(nin[i][0], {DF_F32})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs an F32 input", nn);
        s = bind_output(g, p, nout[i][0], DF_F32, w, h, nn);
        break;
      case NK_SOBEL3:
        if (!need(nin[i][0], {DF_U8})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8 input", nn);
        for (int v : nout[i])
          if (v >= 0 && !s) s = bind_output(g, p, v, DF_S16, w, h, nn);
        break;
      case NK_MAGNITUDE:
      case NK_PHASE:
        if (!need(nin[i][0], {DF_S16}) || !need(nin[i][1], {DF_S16}))
          return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs S16 inputs", nn);
        s = bind_output(g, p, nout[i][0], n->kind == NK_MAGNITUDE ? DF_S16 : DF_U8, w, h, nn);
        break;
      case NK_ADD: {
        if (!need(nin[i][0], {DF_U8, DF_S16}) || !need(nin[i][1], {DF_U8, DF_S16}))
          return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs U8/S16 inputs", nn);
        bool both_u8 = p.vals[nin[i][0]].df == DF_U8 && p.vals[nin[i][1]].df == DF_U8;
        Value& o = p.vals[nout[i][0]];
        int df = (o.is_virtual && o.img->df == DF_VIRT) ? (both_u8 ? DF_U8 : DF_S16) : o.df;
        if (df != DF_U8 && df != DF_S16) return err(g, HVX_ERROR_INVALID_FORMAT, "%s output must be U8 or S16", nn);
        if (df == DF_U8 && !both_u8) return err(g, HVX_ERROR_INVALID_FORMAT, "%s: U8 output needs U8 inputs", nn);
        s = bind_output(g, p, nout[i][0], df, w, h, nn);
        break;
      }
      case NK_MULF:
        if (!need(nin[i][0], {DF_U8, DF_S16}) || !need(nin[i][1], {DF_U8, DF_S16}))
          return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs U8/S16 inputs", nn);
        s = bind_output(g, p, nout[i][0], DF_F32, w, h, nn);
        break;
      case NK_HARRIS:
        for (int v : nin[i])
          if (!need(v, {DF_F32})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs F32 inputs", nn);
        s = bind_output(g, p, nout[i][0], DF_F32, w, h, nn);
        break;
      case NK_THRESHOLD:
        if (!need(nin[i][0], {DF_U8, DF_S16, DF_F32}))
          return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8, S16 or F32 input", nn);
        s = bind_output(g, p, nout[i][0], DF_U8, w, h, nn);
        break;
      case NK_CONVOLVE: {
        if (!need(nin[i][0], {DF_U8})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8 input", nn);
        if (!registry_check(n->conv, T_CONV) && !(n->conv && n->conv->type == T_CONV))
          return err(g, HVX_ERROR_INVALID_REFERENCE, "%s: convolution was released", nn);
        Value& o = p.vals[nout[i][0]];
        int df = (o.is_virtual && o.img->df == DF_VIRT) ? DF_S16 : o.df;
        if (df != DF_U8 && df != DF_S16) return err(g, HVX_ERROR_INVALID_FORMAT, "%s output must be U8 or S16", nn);
        s = bind_output(g, p, nout[i][0], df, w, h, nn);
        break;
      }
      case NK_HISTOGRAM:
        if (!need(nin[i][0], {DF_U8})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8 input", nn);
        s = bind_buffer(g, p, nout[i][0], 4 * (int64_t)n->gp[0], nn);
        break;
      case NK_MINMAX:
      case NK_MINMAXLOC:
        if (!need(nin[i][0], {DF_U8, DF_S16})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8 or S16 input", nn);
        s = bind_buffer(g, p, nout[i][0], n->kind == NK_MINMAX ? kMinMaxBytes : kMMCountBytes, nn);
        if (!s && n->kind == NK_MINMAXLOC && nout[i].size() > 1 && nout[i][1] >= 0)
          s = bind_buffer(g, p, nout[i][1], 16 * (int64_t)n->gp[0], nn);
        break;
      case NK_MEANSTD:
        if (!need(nin[i][0], {DF_U8})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8 input", nn);
        s = bind_buffer(g, p, nout[i][0], kSumsBytes, nn);
        break;
      case NK_EQHIST:
        if (!need(nin[i][0], {DF_U8})) return err(g, HVX_ERROR_INVALID_FORMAT, "%s needs a U8 input", nn);
        s = bind_output(g, p, nout[i][0], DF_U8, w, h, nn);
        break;
      default: return err(g, HVX_ERROR_NOT_SUPPORTED, "unknown node kind");
    }
    if (s) return s;
    // the counts of a global operator are 32-bit
    const bool global = n->kind == NK_HISTOGRAM || n->kind == NK_MINMAX || n->kind == NK_MINMAXLOC ||
                        n->kind == NK_MEANSTD || n->kind == NK_EQHIST;
    if (global && (uint64_t)w * h >= ((uint64_t)1 << 31))
      return err(g, HVX_ERROR_INVALID_DIMENSION, "%s takes images of fewer than 2^31 pixels", nn);
  }

  // ---- 3: lowering to point/local operators ----
  for (int i : order) {
    Node* n = g->nodes[i];
    auto emit = [&](int kind, std::vector<int> ins, int out) {
      LOp o;
      o.kind = kind;
      o.node = i;
      o.nin = (int)ins.size();
      for (int k = 0; k < o.nin; ++k) o.in[k] = ins[k];
      o.out = out;
      o.border = n->border;
      o.bconst = n->bconst;
      o.dval = n->dval;
      o.tv = n->tv;
      o.fv = n->fv;
      o.policy = n->policy;
      o.k = n->k;
      o.conv = n->conv;
      o.expr = &n->expr;
      for (int k = 0; k < 3; ++k) o.gp[k] = n->gp[k];
      op_radius(o, &o.rx, &o.ry);
      p.ops.push_back(o);
    };
    switch (n->kind) {
      case NK_CHANNEL_EXTRACT: emit(OP_CHANNEL_Y, nin[i], nout[i][0]); break;
      case NK_GAUSS3: emit(OP_GAUSS3, nin[i], nout[i][0]); break;
      case NK_GAUSS5: emit(OP_GAUSS5, nin[i], nout[i][0]); break;
      case NK_BOX3: emit(OP_BOX3, nin[i], nout[i][0]); break;
      case NK_DILATE3: emit(OP_DILATE3, nin[i], nout[i][0]); break;
      case NK_ERODE3: emit(OP_ERODE3, nin[i], nout[i][0]); break;
      case NK_MEDIAN3: emit(OP_MEDIAN3, nin[i], nout[i][0]); break;
      case NK_NONLINEAR: emit(OP_NONLINEAR, nin[i], nout[i][0]); break;
      case NK_NONMAX: emit(OP_NONMAX, nin[i], nout[i][0]); break;
      case NK_CUSTOM_POINT: emit(OP_EXPR, nin[i], nout[i][0]); break;
      case NK_CUSTOM_LOCAL: emit(OP_EXPR_LOCAL, nin[i], nout[i][0]); break;
      case NK_BOX5F: emit(OP_BOX5F, nin[i], nout[i][0]); break;
      case NK_SOBEL3:  // two parallel local operators
        if (nout[i][0] >= 0) emit(OP_SOBEL_X, nin[i], nout[i][0]);
        if (nout[i].size() > 1 && nout[i][1] >= 0) emit(OP_SOBEL_Y, nin[i], nout[i][1]);
        break;
      case NK_MAGNITUDE: emit(OP_MAGNITUDE, nin[i], nout[i][0]); break;
      case NK_PHASE: emit(OP_PHASE, nin[i], nout[i][0]); break;
      case NK_ADD: emit(OP_ADD, nin[i], nout[i][0]); break;
      case NK_MULF: emit(OP_MULF, nin[i], nout[i][0]); break;
      case NK_HARRIS: emit(OP_HARRIS, nin[i], nout[i][0]); break;
      case NK_THRESHOLD: emit(OP_THRESHOLD, nin[i], nout[i][0]); break;
      case NK_CONVOLVE: emit(OP_CONVOLVE, nin[i], nout[i][0]); break;
      case NK_HISTOGRAM: emit(OP_HISTOGRAM, nin[i], nout[i][0]); break;
      case NK_MINMAX: emit(OP_MINMAX, nin[i], nout[i][0]); break;
      case NK_MEANSTD: emit(OP_SUMS, nin[i], nout[i][0]); break;
      case NK_MINMAXLOC:  // the counts in one pass, the locations in a second one
        emit(OP_MMCOUNT, nin[i], nout[i][0]);
        if (nout[i].size() > 1 && nout[i][1] >= 0) emit(OP_MMLOCS, {nin[i][0], nout[i][0]}, nout[i][1]);
        break;
      case NK_EQHIST: {
        // histogram and mapping into a buffer of the graph's own, then the
        // mapping applied as a point operator
        Value t;
        t.df = DF_BUF;
        t.w = kEqHistBytes;
        t.h = 1;
        t.is_virtual = true;
        p.vals.push_back(t);
        const int tv = (int)p.vals.size() - 1;
        emit(OP_EQHIST, nin[i], tv);
        emit(OP_LUT, {nin[i][0], tv}, nout[i][0]);
        break;
      }
    }
  }
  p.num_ops = (int)p.ops.size();
  for (size_t o = 0; o < p.ops.size(); ++o) {
    p.vals[p.ops[o].out].producer = (int)o;
    for (int k = 0; k < p.ops[o].nin; ++k) p.vals[p.ops[o].in[k]].consumers.push_back((int)o);
  }

  // ---- 4: dead-computation elimination (Section 5.2.2, Algorithm 1) ----
  // Only non-virtual images are visible after a process call, so an operator
  // is needed exactly when it writes a non-virtual image or writes a virtual
  // one that a needed operator reads.  Liveness is therefore one backward
  // reachability over operators: seed a worklist with every operator whose
  // output is non-virtual, and from each operator taken off the list mark the
  // producers of its virtual inputs.  (A non-virtual image that is also read
  // is a seed itself, so the walk never needs to pass through one.)
  if (g->opt_dce) {
    for (auto& o : p.ops) o.live = false;
    std::vector<int> work;
    for (size_t o = 0; o < p.ops.size(); ++o)
      if (!p.vals[p.ops[o].out].is_virtual) {
        p.ops[o].live = true;
        work.push_back((int)o);
      }
    while (!work.empty()) {
      const LOp& o = p.ops[work.back()];
      work.pop_back();
      for (int k = 0; k < o.nin; ++k) {
        const Value& in = p.vals[o.in[k]];
        if (!in.is_virtual || in.producer < 0 || p.ops[in.producer].live) continue;
        p.ops[in.producer].live = true;
        work.push_back(in.producer);
      }
    }
  }
  // consumer lists and liveness restricted to live operators
  for (auto& v : p.vals) {
    std::vector<int> c;
    for (int o : v.consumers)
      if (p.ops[o].live) c.push_back(o);
    v.consumers = c;
    v.live = (v.producer >= 0 && p.ops[v.producer].live) || !v.consumers.empty();
  }
  p.num_live = 0;
  for (size_t o = 0; o < p.ops.size(); ++o)
    if (p.ops[o].live) {
      p.topo.push_back((int)o);
      ++p.num_live;
    }
  if (p.num_live == 0) return err(g, HVX_ERROR_INVALID_GRAPH, "no operator reaches a non-virtual image");

  // ---- plan choice ----
  // The operator signature keys the tuner's plan choices: it names every
  // live operator with its border and the values it reads and writes, and
  // every value's format, size and kind, so a choice recorded for one graph
  // applies to any graph built the same way.
  {
    std::string key;
    char buf[96];
    snprintf(buf, sizeof buf, "f%d.s%d.c%d:", g->opt_fusion, g->opt_specialize, g->opt_codegen);
    key += buf;
    for (int o : p.topo) {
      const LOp& op = p.ops[o];
      snprintf(buf, sizeof buf, "%d.%d(%d,%d,%d>%d)", op.kind, op.border, op.in[0], op.in[1], op.in[2], op.out);
      key += buf;
    }
    key += "|";
    for (const Value& v : p.vals) {
      snprintf(buf, sizeof buf, "%d.%ux%u%s,", v.df, v.w, v.h, v.is_virtual ? "v" : "");
      key += buf;
    }
    p.op_key = key;
  }
  const TuneEntry* choice = g->plan_choice;
  if (!choice) {
    auto it = g->ctx->tune.find("plan|" + p.op_key);
    if (it != g->ctx->tune.end() && it->second.has_plan) choice = &it->second;
  }

  // ---- 5: grouping ----
  // A global operator's result is complete only once every pixel has been
  // seen, so whatever reads it runs in a later kernel.  The phase of an
  // operator counts the global operators on its longest path from the graph
  // inputs; producer and consumer fuse only within one phase.  (The live
  // operators are in a topological order: nodes in dependency order, each
  // node's operators in their own.)
  std::vector<int> phase(p.ops.size(), 0);
  for (int o : p.topo)
    for (int k = 0; k < p.ops[o].nin; ++k) {
      const int pr = p.vals[p.ops[o].in[k]].producer;
      if (pr >= 0 && p.ops[pr].live) phase[o] = std::max(phase[o], phase[pr] + (is_global_op(p.ops[pr].kind) ? 1 : 0));
    }
  // Fusion on: one group per weakly connected component of live operators
  // of one phase (the location pass of MinMaxLoc alone).  Fusion off: one
  // group per operator ("node by node").
  // A plan choice may cut fusion at some values: their producer and
  // consumers then fuse only through other values.
  std::set<int> cuts;
  if (choice)
    for (int v : choice->cuts)
      if (v >= 0 && v < (int)p.vals.size()) cuts.insert(v);
  std::vector<int> comp(p.ops.size(), -1);
  if (g->opt_fusion) {
    std::vector<int> parent(p.ops.size());
    for (size_t i = 0; i < parent.size(); ++i) parent[i] = (int)i;
    std::function<int(int)> find = [&](int x) { return parent[x] == x ? x : parent[x] = find(parent[x]); };
    for (int o : p.topo) {
      if (p.ops[o].kind == OP_MMLOCS) continue;
      for (int k = 0; k < p.ops[o].nin; ++k) {
        int pr = p.vals[p.ops[o].in[k]].producer;
        if (pr >= 0 && p.ops[pr].live && phase[pr] == phase[o] && !is_global_op(p.ops[pr].kind) &&
            !cuts.count(p.ops[o].in[k]))
          parent[find(o)] = find(pr);
      }
    }
    for (int o : p.topo) comp[o] = find(o);
  } else {
    for (int o : p.topo) comp[o] = o;
  }
  std::map<int, int> gid;
  for (int o : p.topo) {
    if (!gid.count(comp[o])) {
      gid[comp[o]] = (int)p.groups.size();
      p.groups.emplace_back();
      p.groups.back().phase = phase[o];
    }
    p.groups[gid[comp[o]]].ops.push_back(o);
  }
  // inputs/outputs of each group; virtual values crossing groups are materialised
  auto finish_group = [&](Group& gr) {
    std::set<int> ops(gr.ops.begin(), gr.ops.end());
    gr.inputs.clear();
    gr.outputs.clear();
    for (int o : gr.ops) {
      for (int k = 0; k < p.ops[o].nin; ++k) {
        int v = p.ops[o].in[k];
        int pr = p.vals[v].producer;
        if ((pr < 0 || !ops.count(pr)) && std::find(gr.inputs.begin(), gr.inputs.end(), v) == gr.inputs.end())
          gr.inputs.push_back(v);
      }
      int v = p.ops[o].out;
      bool outside = false;
      for (int c : p.vals[v].consumers) outside |= !ops.count(c);
      if (!p.vals[v].is_virtual || outside) gr.outputs.push_back(v);
      if (p.vals[v].is_virtual && outside) p.vals[v].materialize = true;
    }
    // the image size the group runs over (a global operator's output is a
    // buffer: its input gives the size)
    const LOp& o0 = p.ops[gr.ops[0]];
    const Value& sz = p.vals[p.vals[o0.out].df == DF_BUF ? o0.in[0] : o0.out];
    gr.w = sz.w;
    gr.h = sz.h;
  };
  for (auto& gr : p.groups) finish_group(gr);
  // a component too big for one generic kernel is split into single operators
  std::vector<Group> final_groups;
  for (auto& gr : p.groups) {
    int a, b, c;
    bool fast = g->opt_specialize && fast_borders(p, gr) &&
                (match_edge(p, gr, &a, &b, &c) || match_corner(p, gr, &a, &b) || match_gauss5(p, gr, &a, &b));
    std::string why;
    if (!fast && gr.ops.size() > 1) {
      Group probe = gr;
      if (repeat_reads_intermediate(p, gr) || !build_generic(g, p, probe, &why) || probe.footprint > 8) {
        for (int o : gr.ops) {
          Group s;
          s.ops.push_back(o);
          s.phase = gr.phase;
          final_groups.push_back(s);
        }
        continue;
      }
    }
    final_groups.push_back(gr);
  }
  // launch order: every group after the groups whose values it reads (of
  // the groups ready at each step, the one of the earliest phase, then of
  // the earliest first operator)
  {
    std::vector<int> owner(p.ops.size(), -1);
    for (size_t i = 0; i < final_groups.size(); ++i)
      for (int o : final_groups[i].ops) owner[o] = (int)i;
    const size_t n = final_groups.size();
    std::vector<std::set<int>> succ(n);
    std::vector<int> indeg(n, 0);
    for (size_t i = 0; i < n; ++i)
      for (int o : final_groups[i].ops)
        for (int k = 0; k < p.ops[o].nin; ++k) {
          const int pr = p.vals[p.ops[o].in[k]].producer;
          if (pr < 0 || owner[pr] < 0 || owner[pr] == (int)i) continue;
          if (succ[owner[pr]].insert((int)i).second) ++indeg[i];
        }
    std::vector<Group> ordered;
    std::vector<bool> done(n, false);
    for (size_t step = 0; step < n; ++step) {
      int best = -1;
      for (size_t i = 0; i < n; ++i) {
        if (done[i] || indeg[i]) continue;
        const Group& a = final_groups[i];
        if (best < 0 || a.phase < final_groups[best].phase ||
            (a.phase == final_groups[best].phase && a.ops[0] < final_groups[best].ops[0]))
          best = (int)i;
      }
      if (best < 0)
        return err(g, HVX_ERROR_INVALID_GRAPH,
                   "the plan choice for this graph makes its kernels depend on each other in a cycle");
      done[best] = true;
      ordered.push_back(final_groups[best]);
      for (int j : succ[best]) --indeg[j];
    }
    final_groups.swap(ordered);
  }
  p.groups.swap(final_groups);
  p.cuts.assign(cuts.begin(), cuts.end());
  for (auto& v : p.vals) v.materialize = false;
  for (auto& gr : p.groups) finish_group(gr);

  // ---- 6: kernel choice and launch shape ----
  for (auto& gr : p.groups) {
    int in_v = -1, out_v = -1, aux = -1;
    gr.kind = FK_GENERIC;
    if (gr.ops.size() == 1 && is_global_op(p.ops[gr.ops[0]].kind)) {
      // one global operator over an image in memory: the streaming reduction kernels
      gr.kind = FK_GLOBAL;
      gr.v_in = p.ops[gr.ops[0]].in[0];
      gr.v_out = p.ops[gr.ops[0]].out;
      continue;
    }
    if (g->opt_specialize && fast_borders(p, gr)) {
      if (match_edge(p, gr, &in_v, &out_v, &aux)) gr.kind = FK_EDGE;
      else if (match_corner(p, gr, &in_v, &out_v)) gr.kind = FK_CORNER;
      else if (match_gauss5(p, gr, &in_v, &out_v)) gr.kind = FK_GAUSS5;
    }
    if (gr.kind != FK_GENERIC) {
      gr.v_in = in_v;
      gr.v_out = out_v;
      gr.v_aux = aux;
      gr.footprint = gr.kind == FK_CORNER ? 3 : 2;
      continue;
    }
    std::string why;
    if (!build_generic(g, p, gr, &why))
      return err(g, HVX_ERROR_NOT_SUPPORTED, "cannot plan a kernel: %s", why.c_str());
    // the group's own kernel, its operators and formats as constants
    // (Section 6); the interpreter runs the group if it cannot be made
    if (g->opt_codegen && gen_wanted(gr.prog)) {
      GenSource src;
      int tw = 0, th = 0;
      if (choice)
        for (const auto& t : choice->tiles)
          if (t[0] == gr.ops[0]) {
            tw = t[1];
            th = t[2];
          }
      // outputs that no other group reads stream past the caches
      uint32_t stream = 0;
      const std::set<int> own(gr.ops.begin(), gr.ops.end());
      for (size_t i = 0; i < gr.gvals.size(); ++i) {
        if (!gr.prog.vals[i].store) continue;
        bool later = false;
        for (int c : p.vals[gr.gvals[i]].consumers) later |= !own.count(c);
        if (!later) stream |= 1u << i;
      }
      // a chosen tile that does not fit falls back to the default one
      if (!(tw && gen_source(gr.prog, tw, th, stream, &src, &why)) && !gen_source(gr.prog, 0, 0, stream, &src, &why))
        src.text.clear();
      if (!src.text.empty()) gr.gen = gen_compile(src, &why);
      if (gr.gen && src.form == GEN_TILES) p.tiles.push_back({gr.ops[0], src.tw, src.th});
      if (gr.gen) {
        ++p.num_generated;
      } else {
        p.gen_note = why;
        if (getenv("HVX_GEN_LOG")) fprintf(stderr, "hvx: group left to the interpreter: %s\n", why.c_str());
      }
    }
  }

  // byte accounting
  p.alg_bytes = 0;
  p.hbm_bytes = 0;
  p.scratch_bytes = 0;
  for (size_t v = 0; v < p.vals.size(); ++v) {
    const Value& val = p.vals[v];
    int64_t bytes = (int64_t)val.w * val.h * df_bytes(val.df);
    if (!val.is_virtual && val.live) p.alg_bytes += bytes;
    if (val.materialize) p.scratch_bytes += (int64_t)((val.w * df_bytes(val.df) + 63) / 64 * 64) * val.h;
  }
  for (auto& gr : p.groups) {
    for (int v : gr.inputs) p.hbm_bytes += (int64_t)p.vals[v].w * p.vals[v].h * df_bytes(p.vals[v].df);
    for (int v : gr.outputs) p.hbm_bytes += (int64_t)p.vals[v].w * p.vals[v].h * df_bytes(p.vals[v].df);
    if (is_strip_kind(gr.kind)) {
      gr.rows = g->opt_tile ? g->opt_tile : 0;  // 0: tuned or default at schedule time
      gr.xcd = g->opt_xcd;
    }
  }
  g->plan = std::move(pp);
  g->verified = true;
  return HVX_SUCCESS;
}

std::string graph_signature(const Graph* g) {
  std::string s;
  if (!g->plan) return s;
  char buf[160];
  for (const Group& gr : g->plan->groups) {
    snprintf(buf, sizeof buf, "k%d:%ux%u:", gr.kind, gr.w, gr.h);
    s += buf;
    for (int o : gr.ops) {
      const LOp& op = g->plan->ops[o];
      snprintf(buf, sizeof buf, "%d.%d.%u,", op.kind, op.border, op.bconst);
      s += buf;
    }
    s += ";";
  }
  return s;
}

}  // namespace hvx
