// Kernels generated for fused groups: source emission, hipRTC compilation,
// a process-wide cache of code objects and their launch.
//
// A generated tile kernel evaluates the group's operators in stages.  A
// stage is a run of operators that need no barrier between them: each
// thread sweeps the positions of the stage's extent and, at each position,
// evaluates every operator of the stage whose own extent holds it, keeping
// the results in registers.  A value crosses into LDS only when a local
// operator of a later stage reads it at window offsets (or a later stage
// reads it at all); a local operator that reads a value of the current
// stage starts a new stage.  Group inputs that local operators read are
// loaded into LDS with their halo; inputs read only by point operators are
// read from global memory at the pixel itself.  Every window offset, tile
// pitch and LDS offset is a literal, so a read is one LDS access with a
// constant offset.  Tiles whose halo lies inside the image take a body
// without border tests; the others apply each operator's border rule.
#include "codegen.h"

#include <hip/hiprtc.h>

#include <algorithm>
#include <array>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#ifndef HVX_ARCH
#define HVX_ARCH "gfx950"
#endif

namespace hvx {

// the device headers the generated source includes, embedded at build time
extern const int kRtcHeaderCount;
extern const char* const kRtcHeaderNames[];
extern const char* const kRtcHeaderTexts[];

namespace {

constexpr int kGenThreads = 256;
constexpr int kGenLdsBytes = 48 * 1024;
constexpr int kMaxDevices = 64;

bool is_local(int kind) { return !is_point_op(kind) && !is_global_op(kind); }

struct Text {
  std::string s;
  void operator()(const char* fmt, ...) __attribute__((format(printf, 2, 3))) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    int n = vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n >= (int)sizeof buf) {
      std::vector<char> big(n + 1);
      va_start(ap, fmt);
      vsnprintf(big.data(), big.size(), fmt, ap);
      va_end(ap);
      s += big.data();
    } else {
      s += buf;
    }
    s += '\n';
  }
};

std::string fmt(const char* f, ...) __attribute__((format(printf, 1, 2)));
std::string fmt(const char* f, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, f);
  vsnprintf(buf, sizeof buf, f, ap);
  va_end(ap);
  return buf;
}

std::string float_lit(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return fmt("__builtin_bit_cast(float, 0x%08xu)", u);
}

// A Convolve mask that is the outer product of a column and a row of
// integers, m[j][i] = a[j] b[i], as those two factors (b divided by the gcd
// of its entries; every integer factorisation is a multiple of that one).
// Summing each window column with the weights a and then the column sums
// with the weights b gives the same 32-bit wrapped sum as the mask itself,
// since the two double sums are equal as integers.
bool conv_rank_one(const GOp& o, int a[5], int b[5]) {
  const int cols = o.p0, rows = o.p1;
  int j0 = -1;
  for (int j = 0; j < rows && j0 < 0; ++j)
    for (int i = 0; i < cols; ++i)
      if (o.mask[j * cols + i]) j0 = j;
  if (j0 < 0) return false;
  int g = 0;
  for (int i = 0; i < cols; ++i) g = std::gcd(g, std::abs(o.mask[j0 * cols + i]));
  int i0 = -1;
  for (int i = 0; i < cols; ++i) {
    b[i] = o.mask[j0 * cols + i] / g;
    if (b[i] && i0 < 0) i0 = i;
  }
  for (int j = 0; j < rows; ++j) {
    const int m0 = o.mask[j * cols + i0];
    if (m0 % b[i0]) return false;
    a[j] = m0 / b[i0];
    for (int i = 0; i < cols; ++i)
      if (o.mask[j * cols + i] != a[j] * b[i]) return false;
  }
  return true;
}

// column-first costs (4 + 2 rx) column sums of the non-zero weights of a
// plus four sums of those of b, against four sums over the mask's non-zeros
bool separable_pays(const GOp& o, const int a[5], const int b[5]) {
  int na = 0, nb = 0, nm = 0;
  for (int j = 0; j < o.p1; ++j) na += a[j] != 0;
  for (int i = 0; i < o.p0; ++i) nb += b[i] != 0;
  for (int k = 0; k < o.p0 * o.p1; ++k) nm += o.mask[k] != 0;
  return na * (4 + 2 * o.rx) + 4 * nb < 4 * nm;
}

// "0u + c * (unsigned)(e) ..." over the non-zero weights: 32-bit wrapping.
// With `i24` every e lies in [-2^23, 2^23): a weight that is not a power of
// two then multiplies through the 24-bit multiplier (exact, full rate) in
// place of the 32-bit one.
std::string weighted_sum(const int* c, const std::vector<std::string>& e, bool i24) {
  std::string s = "0u";
  for (size_t k = 0; k < e.size(); ++k) {
    if (!c[k]) continue;
    const unsigned m = (unsigned)std::abs(c[k]);
    s += c[k] > 0 ? " + " : " - ";
    if (m == 1) s += "(unsigned)(" + e[k] + ")";
    else if (i24 && (m & (m - 1))) s += "(unsigned)__mul24((int)(" + e[k] + fmt("), %u)", m);
    else s += fmt("%uu * (unsigned)(", m) + e[k] + ")";
  }
  return s;
}

// The operator as a constant the device helpers fold over.
void emit_gop(Text& t, int k, const GOp& o) {
  std::string m, c, kc;
  for (int i = 0; i < kMaxMask; ++i) m += fmt("%s%d", i ? ", " : "", o.mask[i]);
  for (int i = 0; i < kMaxExpr; ++i) c += fmt("%s%d", i ? ", " : "", o.code[i]);
  for (int i = 0; i < kMaxExprConst; ++i) kc += fmt("%s%d", i ? ", " : "", o.kc[i]);
  t("__device__ constexpr GOp gop%d = {%d, %d, {%d, %d, %d}, %d, %d, %s, %d, %d, %d, %d, %d, %d, %s, {%s}, {%s}, {%s}};",
    k, o.kind, o.out, o.in[0], o.in[1], o.in[2], o.border, o.cint, float_lit(o.cf).c_str(), o.rx, o.ry, o.p0, o.p1,
    o.p2, o.p3, float_lit(o.pf).c_str(), m.c_str(), c.c_str(), kc.c_str());
}

// A user kernel's postfix program as one expression (Section 5.1).  The
// arithmetic follows the interpreter's rules: 32-bit wrapping integer
// arithmetic with the result saturated to the output format, or F32 with
// every operation rounded (no contraction).
bool emit_expr(Text& t, int k, const GOp& o, bool local, int out_df, std::string* why) {
  const bool fl = o.p1 != 0;
  std::vector<std::string> st;
  auto pop = [&](std::string* s) {
    if (st.empty()) return false;
    *s = st.back();
    st.pop_back();
    return true;
  };
  if (o.p0 < 1 || o.p0 > kMaxExpr) {
    *why = "malformed user kernel";
    return false;
  }
  for (int i = 0; i < o.p0; ++i) {
    const int op = o.code[i] & 0xFF, arg = o.code[i] >> 8;
    std::string a, b, c;
    bool ok = true;
    switch (op) {
      case X_IN:
      case X_INW: {
        std::string v = local ? (op == X_IN ? std::string("rd(0, 0)") : fmt("rd(%d, %d)", arg % 5 - 2, arg / 5 - 2))
                              : fmt("a%d", arg);
        if (fl) v = ((o.p2 >> (op == X_IN ? arg : 0)) & 1) ? "__int_as_float(" + v + ")" : "(float)(" + v + ")";
        st.push_back(v);
        break;
      }
      case X_CONST:
        if (arg < 0 || arg >= kMaxExprConst) ok = false;
        else st.push_back(fl ? fmt("__int_as_float((int)0x%08xu)", (uint32_t)o.kc[arg]) : fmt("(int)0x%08xu", (uint32_t)o.kc[arg]));
        break;
      case X_ADD:
      case X_SUB:
      case X_MUL:
      case X_DIV:
      case X_MIN:
      case X_MAX:
      case X_GT: {
        ok = pop(&b) && pop(&a);
        if (!ok) break;
        static const char* iname[] = {"gx_add", "gx_sub", "gx_mul", "gx_div"};
        std::string r;
        if (op == X_MIN) r = (fl ? "fminf(" : "min(") + a + ", " + b + ")";
        else if (op == X_MAX) r = (fl ? "fmaxf(" : "max(") + a + ", " + b + ")";
        else if (op == X_GT) r = "((" + a + ") > (" + b + ")" + (fl ? " ? 1.f : 0.f)" : " ? 1 : 0)");
        else if (fl) r = "(" + a + (op == X_ADD ? " + " : op == X_SUB ? " - " : op == X_MUL ? " * " : " / ") + b + ")";
        else r = std::string(iname[op - X_ADD]) + "(" + a + ", " + b + ")";
        st.push_back(r);
        break;
      }
      case X_NEG:
      case X_ABS:
      case X_SQRT:
        ok = pop(&a);
        if (!ok) break;
        if (op == X_NEG) st.push_back(fl ? "(-(" + a + "))" : "gx_neg(" + a + ")");
        else if (op == X_ABS) st.push_back(fl ? "fabsf(" + a + ")" : "gx_abs(" + a + ")");
        else if (fl) st.push_back("__builtin_sqrtf(" + a + ")");
        else ok = false;
        break;
      case X_CLAMP:
        ok = pop(&c) && pop(&b) && pop(&a);
        if (ok) st.push_back(fl ? "fminf(fmaxf(" + a + ", " + b + "), " + c + ")" : "min(max(" + a + ", " + b + "), " + c + ")");
        break;
      case X_SEL:
        ok = pop(&c) && pop(&b) && pop(&a);
        if (ok) st.push_back("((" + a + ") != " + (fl ? "0.f" : "0") + " ? (" + b + ") : (" + c + "))");
        break;
      default: ok = false;
    }
    if (!ok) {
      *why = "malformed user kernel";
      return false;
    }
  }
  if (st.size() != 1) {
    *why = "malformed user kernel";
    return false;
  }
  if (local) t("template <class RD> __device__ __forceinline__ int gx_expr%d(const RD& rd) {", k);
  else t("__device__ __forceinline__ int gx_expr%d(int a0, int a1, int a2) {", k);
  t("#pragma clang fp contract(off)");
  if (fl) {
    t("  const float r = %s;", st[0].c_str());
    t("  return __float_as_int(r);");
  } else {
    t("  const int r = %s;", st[0].c_str());
    t(out_df == DF_U8 ? "  return min(max(r, 0), 255);" : "  return min(max(r, -32768), 32767);");
  }
  t("}");
  return true;
}

void emit_prelude(Text& t, const GProg& P, std::string* why, bool* ok) {
  t("namespace __hip_internal {}");
  t("using namespace __hip_internal;");
  t("#include \"dev_generic.hpp\"");
  t("#include \"gen_abi.h\"");
  t("namespace hvx {");
  t("__device__ __forceinline__ int gx_add(int a, int b) { return (int)((uint32_t)a + (uint32_t)b); }");
  t("__device__ __forceinline__ int gx_sub(int a, int b) { return (int)((uint32_t)a - (uint32_t)b); }");
  t("__device__ __forceinline__ int gx_mul(int a, int b) { return (int)((uint32_t)a * (uint32_t)b); }");
  t("__device__ __forceinline__ int gx_neg(int a) { return (int)(0u - (uint32_t)a); }");
  t("__device__ __forceinline__ int gx_abs(int a) { return a < 0 ? gx_neg(a) : a; }");
  t("__device__ __forceinline__ int gx_div(int x, int y) { return y == 0 ? 0 : (y == -1 ? gx_neg(x) : x / y); }");
  // a value's LDS tile read under an operator's border rule (edge tiles)
  t("template <int BORDER>");
  t("__device__ __forceinline__ int gx_rd(const int32_t* L, int rw, int ey, int ex, int tx0, int ty0, int W, int H,");
  t("                                    int x, int y, int cval) {");
  t("  if (BORDER != B_REPEAT && (x < 0 || y < 0 || x >= W || y >= H)) {");
  t("    if (BORDER == B_CONSTANT) return cval;");
  t("    if (BORDER == B_MIRROR) {");
  t("      x = mirror_pos(x, W);");
  t("      y = mirror_pos(y, H);");
  t("    }");
  t("    x = min(max(x, 0), W - 1);");
  t("    y = min(max(y, 0), H - 1);");
  t("  }");
  t("  return L[(y - ty0 + ey) * rw + (x - tx0 + ex)];");
  t("}");
  // the image of a batch that work-group `blk` belongs to: the last whose
  // first work-group is at or before it (a uniform binary search)
  t("__device__ __forceinline__ int gx_batch_image(const GenBatchImage* imgs, int n, int blk) {");
  t("  int lo = 0, hi = n - 1;");
  t("  while (lo < hi) {");
  t("    const int mid = (lo + hi + 1) >> 1;");
  t("    if (imgs[mid].block0 <= blk) lo = mid;");
  t("    else hi = mid - 1;");
  t("  }");
  t("  return lo;");
  t("}");
  // four elements of a row from x on; zero outside the image (edge tiles)
  t("__device__ __forceinline__ void gx_load4_edge(int df, const void* base, int64_t pitch, int x, int y, int W, int H,");
  t("                                              int v[4]) {");
  t("#pragma unroll");
  t("  for (int q = 0; q < 4; ++q)");
  t("    v[q] = (y >= 0 && y < H && x + q >= 0 && x + q < W) ? gload(df, base, pitch, x + q, y) : 0;");
  t("}");
  // element j of a 16-byte chunk of a row in format DF (int bits)
  t("template <int DF>");
  t("__device__ __forceinline__ int gx_elem(const uint4& d, int j) {");
  t("  const int bpp = DF == DF_U8 ? 1 : ((DF == DF_S16 || DF == DF_UYVY) ? 2 : 4);");
  t("  const int k = j * bpp / 4, sh = (j * bpp % 4) * 8;");
  t("  const uint32_t w = k == 0 ? d.x : (k == 1 ? d.y : (k == 2 ? d.z : d.w));");
  t("  if (DF == DF_U8) return (int)((w >> sh) & 0xFFu);");
  t("  if (DF == DF_S16) return (int)(int16_t)(uint16_t)(w >> sh);");
  t("  if (DF == DF_UYVY) return (int)((w >> sh) & 0xFFFFu);");
  t("  return (int)w;");
  t("}");
  for (int k = 0; k < P.nops; ++k) {
    emit_gop(t, k, P.ops[k]);
    const GOp& o = P.ops[k];
    if (o.kind == OP_EXPR || o.kind == OP_EXPR_LOCAL)
      if (!emit_expr(t, k, o, o.kind == OP_EXPR_LOCAL, P.vals[o.out].df, why)) *ok = false;
  }
  t("}  // namespace hvx");
  t("using namespace hvx;");
}

// ---- the point form ----------------------------------------------------------

bool emit_points(const GProg& P, uint32_t stream, GenSource* out, std::string* why) {
  Text t;
  bool ok = true;
  emit_prelude(t, P, why, &ok);
  if (!ok) return false;
  t("extern \"C\" __global__ __launch_bounds__(%d) void hvx_gen(const GProg* __restrict__ P, const IOTable io0,",
    kGenThreads);
  t("                                                           const GenBatchImage* __restrict__ imgs, int nimg,");
  t("                                                           uint32_t* __restrict__ ws) {");
  // one image (the program's size), or one image of a batch of images
  t("  IOTable io;");
  t("  int W, H, blk = (int)blockIdx.x;");
  t("  if (nimg == 0) {");
  t("    io = io0;");
  t("    W = P->w;");
  t("    H = P->h;");
  t("  } else {");
  t("    const int i = gx_batch_image(imgs, nimg, blk);");
  t("    io = imgs[i].io;");
  t("    W = imgs[i].w;");
  t("    H = imgs[i].h;");
  t("    blk -= imgs[i].block0;");
  t("  }");
  t("  const int bx = (W + 1023) >> 10;");
  t("  const int y = blk / bx;");
  t("  const int x = ((blk - y * bx) * %d + (int)threadIdx.x) * 4;", kGenThreads);
  t("  if (y >= H || x >= W) return;");
  std::vector<int> read(P.nvals, 0);
  for (int k = 0; k < P.nops; ++k)
    for (int i = 0; i < 3; ++i)
      if (P.ops[k].in[i] >= 0) read[P.ops[k].in[i]] = 1;
  for (int v = 0; v < P.nvals; ++v) {
    const GVal& gv = P.vals[v];
    if (!gv.input || !read[v] || gv.df == DF_BUF) continue;
    t("  int v%d[4];", v);
    t("  load4(%d, (const uint8_t*)io.ptr[%d] + (size_t)y * io.pitch[%d], x, W, v%d);", gv.df, gv.io, gv.io, v);
  }
  for (int k = 0; k < P.nops; ++k) {
    const GOp& o = P.ops[k];
    const GVal& ov = P.vals[o.out];
    t("  int v%d[4];", o.out);
    t("#pragma unroll");
    t("  for (int q = 0; q < 4; ++q) {");
    auto in = [&](int i) { return o.in[i] >= 0 && P.vals[o.in[i]].df != DF_BUF ? fmt("v%d[q]", o.in[i]) : std::string("0"); };
    if (o.kind == OP_LUT)
      t("    v%d[q] = ((const uint8_t*)io.ptr[%d])[%d + (v%d[q] & 0xFF)];", o.out, P.vals[o.in[1]].io, 256 * 4, o.in[0]);
    else if (o.kind == OP_EXPR)
      t("    v%d[q] = gx_expr%d(%s, %s, %s);", o.out, k, in(0).c_str(), in(1).c_str(), in(2).c_str());
    else
      t("    v%d[q] = point_eval(gop%d, %d, %s, %s, %s, %s);", o.out, k, ov.df,
        P.vals[o.in[0]].df == DF_F32 ? "true" : "false", in(0).c_str(), in(1).c_str(), in(2).c_str());
    t("  }");
    if (ov.store)
      t("  store4<%s>(%d, (uint8_t*)io.ptr[%d] + (size_t)y * io.pitch[%d], x, W, v%d);",
        (stream >> o.out) & 1 ? "true" : "false", ov.df, ov.io, ov.io, o.out);
  }
  t("}");
  out->text = t.s;
  out->form = GEN_POINTS;
  out->tw = out->th = 0;
  out->red = false;
  out->lds_words = 0;
  return true;
}

// ---- the tile form -----------------------------------------------------------

enum Src { S_REG = 1, S_LDS, S_GLB };

struct Layout {
  int nstages = 0;
  std::vector<int> op_stage;
  std::vector<int> stage_ev, stage_eh;  // vertical / horizontal extent of each stage's sweep
  std::vector<int> def_stage, last_lds, needs_lds, producer, lds_off;
  std::vector<int> eh;  // horizontal extent of each value: a multiple of 4
  std::vector<std::array<int, 3>> src;
  int lds_words = 0;
  // The border rule the local operators reading a value apply to it, as
  // (mode, constant bits).  When every such value has one rule, edge tiles
  // hold each value's positions outside the image resolved by that rule and
  // run the interior code; otherwise they read through each operator's rule.
  std::vector<int> bmode, bconst;
  bool resolved = true;
};

int round4(int x) { return (x + 3) / 4 * 4; }

void plan_stages(const GProg& P, Layout& L) {
  const int nv = P.nvals, no = P.nops;
  L.op_stage.assign(no, 0);
  L.def_stage.assign(nv, -1);
  L.producer.assign(nv, -1);
  L.needs_lds.assign(nv, 0);
  L.last_lds.assign(nv, -2);
  L.src.assign(no, {0, 0, 0});
  int cur = 0;
  for (int k = 0; k < no; ++k) {
    const GOp& o = P.ops[k];
    bool reads_cur = false;
    if (is_local(o.kind))
      for (int i = 0; i < 3; ++i)
        if (o.in[i] >= 0 && L.producer[o.in[i]] >= 0 && L.def_stage[o.in[i]] == cur) reads_cur = true;
    if (reads_cur) ++cur;
    L.op_stage[k] = cur;
    L.producer[o.out] = k;
    L.def_stage[o.out] = cur;
  }
  L.nstages = cur + 1;
  // reads: local operators read LDS; point operators and reductions read
  // registers within a stage, LDS across stages, group inputs where they are
  for (int k = 0; k < no; ++k) {
    const GOp& o = P.ops[k];
    for (int i = 0; i < 3; ++i) {
      const int v = o.in[i];
      if (v < 0 || P.vals[v].df == DF_BUF) continue;
      if (is_local(o.kind)) {
        L.src[k][i] = S_LDS;
        L.needs_lds[v] = 1;
      } else if (L.producer[v] >= 0) {
        L.src[k][i] = L.def_stage[v] == L.op_stage[k] ? S_REG : S_LDS;
        if (L.src[k][i] == S_LDS) L.needs_lds[v] = 1;
      }
    }
  }
  for (int k = 0; k < no; ++k) {
    const GOp& o = P.ops[k];
    for (int i = 0; i < 3; ++i) {
      const int v = o.in[i];
      if (v < 0 || P.vals[v].df == DF_BUF) continue;
      if (L.producer[v] < 0 && !is_local(o.kind)) L.src[k][i] = L.needs_lds[v] ? S_LDS : S_GLB;
      if (L.src[k][i] == S_LDS) L.last_lds[v] = std::max(L.last_lds[v], L.op_stage[k]);
    }
  }
  // Horizontal extents, consumers first: interior tiles evaluate four
  // horizontally adjacent pixels per thread, so every operator runs over a
  // horizontal extent that is a multiple of 4 (the extra columns are
  // computed like any other), and its input must then hold that extent plus
  // the operator's radius, again rounded up to a multiple of 4.
  L.eh.assign(nv, 0);
  for (int k = no - 1; k >= 0; --k) {
    const GOp& o = P.ops[k];
    const int need = (is_global_op(o.kind) ? 0 : L.eh[o.out]) + (is_local(o.kind) ? o.rx : 0);
    for (int i = 0; i < 3; ++i)
      if (o.in[i] >= 0) L.eh[o.in[i]] = std::max(L.eh[o.in[i]], round4(need));
  }
  L.bmode.assign(nv, -1);
  L.bconst.assign(nv, 0);
  for (int k = 0; k < no; ++k) {
    const GOp& o = P.ops[k];
    if (!is_local(o.kind)) continue;
    const int v = o.in[0];
    uint32_t c = (uint32_t)o.cint;  // the border constant as the input's element bits
    if (P.vals[v].df == DF_F32) memcpy(&c, &o.cf, 4);
    const int mode = o.border == B_UNDEFINED ? B_REPLICATE : o.border;
    const int cb = mode == B_CONSTANT ? (int)c : 0;
    if (L.bmode[v] >= 0 && (L.bmode[v] != mode || L.bconst[v] != cb)) L.resolved = false;
    // REPEAT reads periodic copies: only a group input's load provides them
    if (mode == B_REPEAT && L.producer[v] >= 0) L.resolved = false;
    L.bmode[v] = mode;
    L.bconst[v] = cb;
  }
  L.stage_ev.assign(L.nstages, 0);
  L.stage_eh.assign(L.nstages, 0);
  for (int k = 0; k < no; ++k) {
    const GOp& o = P.ops[k];
    if (is_global_op(o.kind)) continue;
    L.stage_ev[L.op_stage[k]] = std::max(L.stage_ev[L.op_stage[k]], P.vals[o.out].ext);
    L.stage_eh[L.op_stage[k]] = std::max(L.stage_eh[L.op_stage[k]], L.eh[o.out]);
  }
}

// LDS geometry of a value kept on chip: rows of `rw` words, image column x
// of the tile at column x - tx0 + co, image row y at row y - ty0 + e (its
// vertical extent).  A group input is loaded in whole 16-byte chunks of its
// rows, so its rows start at a 16-byte boundary of the image row before the
// halo.  Every row width and column offset is a multiple of 4 words.
int input_cols(const GVal& v, int eh) {
  const int bpp = df_bytes(v.df);
  return ((eh * bpp + 15) / 16 * 16) / bpp;
}

void value_geometry(const GProg& P, const Layout& L, int v, int tw, int* rw, int* co) {
  const GVal& gv = P.vals[v];
  *co = gv.input ? input_cols(gv, L.eh[v]) : L.eh[v];
  *rw = tw + 2 * *co;
}

// First-fit LDS blocks; two values share words only if one is last read in
// a stage before the other is written.  Blocks start at 16-byte boundaries.
int place_lds(const GProg& P, Layout& L, int tw, int th) {
  const int nv = P.nvals;
  L.lds_off.assign(nv, -1);
  std::vector<int> order;
  for (int v = 0; v < nv; ++v)
    if (L.needs_lds[v]) order.push_back(v);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return L.def_stage[a] < L.def_stage[b]; });
  std::vector<std::array<int, 4>> blocks;  // offset, size, first stage, last stage
  int top = 0;
  for (int v : order) {
    int rw, co;
    value_geometry(P, L, v, tw, &rw, &co);
    const int sz = round4(rw * (th + 2 * P.vals[v].ext));
    const int d = L.def_stage[v], l = std::max(L.last_lds[v], d);
    std::vector<std::array<int, 2>> busy;
    for (auto& b : blocks)
      if (!(b[3] < d || l < b[2])) busy.push_back({b[0], b[1]});
    std::sort(busy.begin(), busy.end());
    int pos = 0;
    for (auto& b : busy) {
      if (pos + sz <= b[0]) break;
      pos = std::max(pos, b[0] + b[1]);
    }
    L.lds_off[v] = pos;
    top = std::max(top, pos + sz);
    blocks.push_back({pos, sz, d, l});
  }
  L.lds_words = top;
  return top;
}

// Load group input v into LDS.  Interior tiles read whole 16-byte chunks
// (every chunk holds a byte of the extent, so it lies inside the row's
// pitch, a multiple of 64 bytes): one vector load per chunk, all of a
// thread's loads issued before the first LDS write.  (Loading four elements
// per lane instead, so that the 16-byte LDS writes of consecutive lanes are
// consecutive, measured slower overall.)  Edge tiles read element by element
// inside the image (or the periodic copies under REPEAT).
void emit_load(Text& t, const GProg& P, const Layout& L, int v, int TW, int TH) {
  const GVal& gv = P.vals[v];
  const int e = gv.ext, eh = L.eh[v], bpp = df_bytes(gv.df);
  int rw, co;
  value_geometry(P, L, v, TW, &rw, &co);
  const int rows = TH + 2 * e, epc = 16 / bpp, cpr = rw / epc, nch = cpr * rows;
  const int kc = (nch + kGenThreads - 1) / kGenThreads;
  const int off = L.lds_off[v];
  t("  {  // load value %d: %d rows of %d columns (halo %d rows, %d columns)", v, rows, rw, e, eh);
  t("    const uint8_t* base = (const uint8_t*)io.ptr[%d];", gv.io);
  t("    const int64_t pitch = io.pitch[%d];", gv.io);
  t("    if constexpr (IN) {");
  t("      uint4 d[%d];", kc);
  t("#pragma unroll");
  t("      for (int k = 0; k < %d; ++k) {", kc);
  t("        const int c = (int)threadIdx.x + k * %d;", kGenThreads);
  t("        if (c < %d) {", nch);
  t("          const int row = c / %d, q = c - row * %d;", cpr, cpr);
  t("          d[k] = *(const uint4*)(base + (size_t)(ty0 - %d + row) * pitch + (size_t)(tx0 - %d) * %d + q * 16);", e,
    co, bpp);
  t("        }");
  t("      }");
  t("#pragma unroll");
  t("      for (int k = 0; k < %d; ++k) {", kc);
  t("        const int c = (int)threadIdx.x + k * %d;", kGenThreads);
  t("        if (c < %d) {", nch);
  t("          const int row = c / %d, q = c - row * %d;", cpr, cpr);
  t("          gx_i4* dst = (gx_i4*)(L + %d + row * %d + q * %d);", off, rw, epc);
  t("#pragma unroll");
  t("          for (int j = 0; j < %d; j += 4)", epc);
  t("            dst[j / 4] = gx_i4{gx_elem<%d>(d[k], j), gx_elem<%d>(d[k], j + 1), gx_elem<%d>(d[k], j + 2),", gv.df,
    gv.df, gv.df);
  t("                                   gx_elem<%d>(d[k], j + 3)};", gv.df);
  t("        }");
  t("      }");
  t("    } else {");
  t("      for (int i = (int)threadIdx.x; i < %d; i += %d) {", rw * rows, kGenThreads);
  t("        const int ly = i / %d, lx = i - ly * %d;", rw, rw);
  t("        int x = tx0 - %d + lx, y = ty0 - %d + ly;", co, e);
  t("        if (lx < %d || lx >= %d) continue;  // outside the extent", co - eh, co + TW + eh);
  if (gv.wrap) {
    t("        L[%d + i] = gload(%d, base, pitch, repeat_pos(x, W), repeat_pos(y, H));", off, gv.df);
  } else if (L.resolved) {
    // positions outside the image take the border rule of the operators reading the value
    t("        if (x < 0 || y < 0 || x >= W || y >= H) {");
    if (L.bmode[v] == B_CONSTANT) {
      t("          L[%d + i] = (int)0x%08xu;", off, (uint32_t)L.bconst[v]);
      t("          continue;");
    } else if (L.bmode[v] == B_MIRROR) {
      t("          x = mirror_pos(x, W);");
      t("          y = mirror_pos(y, H);");
    }
    t("          x = min(max(x, 0), W - 1);");
    t("          y = min(max(y, 0), H - 1);");
    t("        }");
    t("        L[%d + i] = gload(%d, base, pitch, x, y);", off, gv.df);
  } else {
    t("        if (x >= 0 && y >= 0 && x < W && y < H) L[%d + i] = gload(%d, base, pitch, x, y);", off, gv.df);
  }
  t("      }");
  t("    }");
  t("  }");
}

// Edge tiles: the positions of value v outside the image, resolved by the
// border rule of the operators reading it from the positions inside (which
// lie in the value's tile: a border rule maps a position to one within the
// value's extent of the image's edge).
void emit_fill(Text& t, const GProg& P, const Layout& L, int v, int TW, int TH) {
  const int e = P.vals[v].ext, eh = L.eh[v];
  int rw, co;
  value_geometry(P, L, v, TW, &rw, &co);
  const int rows = TH + 2 * e, off = L.lds_off[v];
  t("    for (int i = (int)threadIdx.x; i < %d; i += %d) {  // border of value %d", rw * rows, kGenThreads, v);
  t("      const int ly = i / %d, lx = i - ly * %d;", rw, rw);
  t("      int x = tx0 - %d + lx, y = ty0 - %d + ly;", co, e);
  t("      if (lx < %d || lx >= %d || (x >= 0 && y >= 0 && x < W && y < H)) continue;", co - eh, co + TW + eh);
  if (L.bmode[v] == B_CONSTANT) {
    t("      L[%d + i] = (int)0x%08xu;", off, (uint32_t)L.bconst[v]);
  } else {
    if (L.bmode[v] == B_MIRROR) {
      t("      x = mirror_pos(x, W);");
      t("      y = mirror_pos(y, H);");
    }
    t("      x = min(max(x, 0), W - 1);");
    t("      y = min(max(y, 0), H - 1);");
    t("      L[%d + i] = L[%d + (y - ty0 + %d) * %d + (x - tx0 + %d)];", off, off, e, rw, co);
  }
  t("    }");
}

// The sweeps of one stage.  Edge tiles (1 px per thread) skip positions
// outside the image and read windows through each operator's border rule.
// Interior tiles take groups of four horizontally adjacent pixels per
// thread: a local operator's window comes from LDS as 16-byte reads (three
// per window row), LDS values move four words at a time, and outputs are
// stored four pixels at a time.
struct StageEmitter {
  Text& t;
  const GProg& P;
  const Layout& L;
  int TW, TH;
  int* slot;
  uint32_t stream;  // values no later kernel reads: non-temporal stores

  void geometry(int v, int* rw, int* co) const { value_geometry(P, L, v, TW, rw, co); }

  // LDS index of value v at the sweep position (+ constant offsets)
  std::string lds_index(int v, int ES_V, int ES_H, const char* dx, const char* dy) const {
    int rw, co;
    geometry(v, &rw, &co);
    return fmt("%d + (ly + %d + %s) * %d + (lx + %d + %s)", L.lds_off[v], P.vals[v].ext - ES_V, dy, rw, co - ES_H, dx);
  }

  void one_pixel(int s) {
    const int ESV = L.stage_ev[s], ESH = L.stage_eh[s];
    const int RW = TW + 2 * ESH, RH = TH + 2 * ESV;
    bool need_own = false;
    for (int k = 0; k < P.nops; ++k)
      if (L.op_stage[k] == s && (is_reduce_op(P.ops[k].kind) || P.vals[P.ops[k].out].store)) need_own = true;
    t("    for (int i = (int)threadIdx.x; i < %d; i += %d) {", RW * RH, kGenThreads);
    t("      const int ly = i / %d, lx = i - ly * %d;", RW, RW);
    t("      const int x = tx0 - %d + lx, y = ty0 - %d + ly;", ESH, ESV);
    t("      if (x < 0 || y < 0 || x >= W || y >= H) continue;");
    if (need_own) t("      const bool own = lx >= %d && lx < %d && ly >= %d && ly < %d;", ESH, ESH + TW, ESV, ESV + TH);
    for (int k = 0; k < P.nops; ++k) {
      if (L.op_stage[k] != s) continue;
      const GOp& o = P.ops[k];
      auto at = [&](int i) -> std::string {
        const int v = o.in[i];
        if (v < 0 || P.vals[v].df == DF_BUF) return "0";
        switch (L.src[k][i]) {
          case S_REG: return fmt("v%d", v);
          case S_GLB: return fmt("gload(%d, io.ptr[%d], io.pitch[%d], x, y)", P.vals[v].df, P.vals[v].io, P.vals[v].io);
          default: return "L[" + lds_index(v, ESV, ESH, "0", "0") + "]";
        }
      };
      if (is_reduce_op(o.kind)) {
        t("      if (own) red_add(rs, %d, gop%d, %s);", (*slot)++, k, at(0).c_str());
        continue;
      }
      const GVal& ov = P.vals[o.out];
      const int EV = ov.ext, EH = L.eh[o.out];
      t("      int v%d = 0;", o.out);
      t("      if (lx >= %d && lx < %d && ly >= %d && ly < %d) {", ESH - EH, ESH + EH + TW, ESV - EV, ESV + EV + TH);
      if (is_local(o.kind)) {
        const int v = o.in[0];
        int rw, co;
        geometry(v, &rw, &co);
        uint32_t cval = (uint32_t)o.cint;  // the border constant as the input's element bits
        if (P.vals[v].df == DF_F32) memcpy(&cval, &o.cf, 4);
        t("        auto rd = [&](int dx, int dy) -> int {");
        t("          return gx_rd<%d>(L + %d, %d, %d, %d, tx0, ty0, W, H, x + dx, y + dy, (int)0x%08xu);", o.border,
          L.lds_off[v], rw, P.vals[v].ext, co, cval);
        t("        };");
        if (o.kind == OP_EXPR_LOCAL) t("        v%d = gx_expr%d(rd);", o.out, k);
        else t("        v%d = local_eval<%s>(gop%d, %d, rd);", o.out, o.kind == OP_NONLINEAR ? "true" : "false", k, ov.df);
      } else if (o.kind == OP_LUT) {
        t("        v%d = ((const uint8_t*)io.ptr[%d])[%d + (%s & 0xFF)];", o.out, P.vals[o.in[1]].io, 256 * 4,
          at(0).c_str());
      } else if (o.kind == OP_EXPR) {
        t("        v%d = gx_expr%d(%s, %s, %s);", o.out, k, at(0).c_str(), at(1).c_str(), at(2).c_str());
      } else {
        t("        v%d = point_eval(gop%d, %d, %s, %s, %s, %s);", o.out, k, ov.df,
          P.vals[o.in[0]].df == DF_F32 ? "true" : "false", at(0).c_str(), at(1).c_str(), at(2).c_str());
      }
      if (L.needs_lds[o.out]) t("        L[%s] = v%d;", lds_index(o.out, ESV, ESH, "0", "0").c_str(), o.out);
      if (ov.store) t("        if (own) gstore(%d, io.ptr[%d], io.pitch[%d], x, y, v%d);", ov.df, ov.io, ov.io, o.out);
      t("      }");
    }
    t("    }");
  }

  void four_pixels(int s, bool edge) {
    const int ESV = L.stage_ev[s], ESH = L.stage_eh[s];
    const int GR = (TW + 2 * ESH) / 4, RH = TH + 2 * ESV;
    bool need_own = false;
    for (int k = 0; k < P.nops; ++k)
      if (L.op_stage[k] == s && (is_reduce_op(P.ops[k].kind) || P.vals[P.ops[k].out].store)) need_own = true;
    t("    for (int i = (int)threadIdx.x; i < %d; i += %d) {", GR * RH, kGenThreads);
    t("      const int ly = i / %d, lx = (i - ly * %d) * 4;", GR, GR);
    t("      const int x = tx0 - %d + lx, y = ty0 - %d + ly;", ESH, ESV);
    if (need_own) t("      const bool own = lx >= %d && lx < %d && ly >= %d && ly < %d;", ESH, ESH + TW, ESV, ESV + TH);
    for (int k = 0; k < P.nops; ++k) {
      if (L.op_stage[k] != s) continue;
      const GOp& o = P.ops[k];
      // four elements of input i at the position: an array name
      auto at4 = [&](int i) -> std::string {
        const int v = o.in[i];
        if (v < 0 || P.vals[v].df == DF_BUF) return "gx_zero4";
        const std::string n = fmt("a%d_%d", k, i);
        switch (L.src[k][i]) {
          case S_REG: return fmt("v%d", v);
          case S_GLB:
            t("        int %s[4];", n.c_str());
            if (edge)
              t("        gx_load4_edge(%d, io.ptr[%d], io.pitch[%d], x, y, W, H, %s);", P.vals[v].df, P.vals[v].io,
                P.vals[v].io, n.c_str());
            else
              t("        load4(%d, (const uint8_t*)io.ptr[%d] + (size_t)y * io.pitch[%d], x, W, %s);", P.vals[v].df,
                P.vals[v].io, P.vals[v].io, n.c_str());
            return n;
          default: {
            t("        int %s[4];", n.c_str());
            t("        { const gx_i4 q = gx_ld4(L + %s); %s[0] = q.x; %s[1] = q.y; %s[2] = q.z; %s[3] = q.w; }",
              lds_index(v, ESV, ESH, "0", "0").c_str(), n.c_str(), n.c_str(), n.c_str(), n.c_str());
            return n;
          }
        }
      };
      if (is_reduce_op(o.kind)) {
        t(edge ? "      if (own && y < H) {" : "      if (own) {");
        const std::string a = at4(0);
        t("#pragma unroll");
        if (edge)
          t("        for (int q = 0; q < 4; ++q) if (x + q < W) red_add(rs, %d, gop%d, %s[q]);", (*slot)++, k, a.c_str());
        else
          t("        for (int q = 0; q < 4; ++q) red_add(rs, %d, gop%d, %s[q]);", (*slot)++, k, a.c_str());
        t("      }");
        continue;
      }
      const GVal& ov = P.vals[o.out];
      const int EV = ov.ext, EH = L.eh[o.out];
      t("      int v%d[4] = {0, 0, 0, 0};", o.out);
      t("      if (lx >= %d && lx < %d && ly >= %d && ly < %d) {", ESH - EH, ESH + EH + TW, ESV - EV, ESV + EV + TH);
      if (is_local(o.kind)) {
        const int v = o.in[0], R = o.ry;
        int rw, co;
        geometry(v, &rw, &co);
        // window row j: input row y - R + j, columns x - 4 .. x + 7
        t("        int w[%d][12];", 2 * R + 1);
        t("#pragma unroll");
        t("        for (int j = 0; j < %d; ++j) {", 2 * R + 1);
        const std::string dy = fmt("(j - %d)", R);
        t("          const int32_t* r = L + %s;", lds_index(v, ESV, ESH, "-4", dy.c_str()).c_str());
        t("#pragma unroll");
        t("          for (int c = 0; c < 3; ++c) {");
        t("            const gx_i4 q = gx_ld4(r + 4 * c);");
        t("            w[j][4 * c] = q.x; w[j][4 * c + 1] = q.y; w[j][4 * c + 2] = q.z; w[j][4 * c + 3] = q.w;");
        t("          }");
        t("        }");
        int ca[5], cb[5];
        const int vdf = P.vals[v].df;
        if (o.kind == OP_CONVOLVE && (vdf == DF_U8 || vdf == DF_S16) && conv_rank_one(o, ca, cb) &&
            separable_pays(o, ca, cb)) {
          // column sums first (columns x - rx .. x + 3 + rx), shared by the
          // four outputs; the mask is flipped as in the operator's definition
          // (inputs are U8 or S16; a column sum stays within 24 bits when
          // the sum of |a| times the input's largest magnitude does)
          const int rx = o.rx, ry = o.ry;
          long long bound = 0;
          for (int j = 0; j < o.p1; ++j) bound += std::abs(ca[j]);
          bound *= vdf == DF_U8 ? 255 : 32768;
          for (int c = 4 - rx; c <= 7 + rx; ++c) {
            std::vector<std::string> e;
            for (int j = -ry; j <= ry; ++j) e.push_back(fmt("w[%d][%d]", R - j, c));
            t("        const unsigned cs%d = %s;", c, weighted_sum(ca, e, true).c_str());
          }
          for (int q = 0; q < 4; ++q) {
            std::vector<std::string> e;
            for (int i = -rx; i <= rx; ++i) e.push_back(fmt("cs%d", 4 + q - i));
            t("        {");
            t("          const int s = (int)(%s);", weighted_sum(cb, e, bound < (1 << 23)).c_str());
            t("          const int d = s >= 0 ? (s >> %d) : -((-s) >> %d);", o.p2, o.p2);
            t("          v%d[%d] = %s(d);", o.out, q, ov.df == DF_U8 ? "sat_u8" : "sat_s16");
            t("        }");
          }
        } else {
        t("        const int (*wp)[12] = w;");
        t("#pragma unroll");
        t("        for (int q = 0; q < 4; ++q) {");
        if (o.kind == OP_EXPR_LOCAL) {
          t("          v%d[q] = gx_expr%d([&](int dx, int dy) { return wp[%d + dy][4 + q + dx]; });", o.out, k, R);
        } else {
          t("          switch (q) {");
          for (int q = 0; q < 4; ++q)
            t("            case %d: v%d[%d] = local_eval<%s>(gop%d, %d, WinRd<%d, %d>{wp}); break;", q, o.out, q,
              o.kind == OP_NONLINEAR ? "true" : "false", k, ov.df, R, q);
          t("          }");
        }
        t("        }");
        }
      } else if (o.kind == OP_LUT) {
        const std::string a = at4(0);
        t("#pragma unroll");
        t("        for (int q = 0; q < 4; ++q) v%d[q] = ((const uint8_t*)io.ptr[%d])[%d + (%s[q] & 0xFF)];", o.out,
          P.vals[o.in[1]].io, 256 * 4, a.c_str());
      } else {
        const std::string a = at4(0), b = at4(1), c = at4(2);
        t("#pragma unroll");
        if (o.kind == OP_EXPR)
          t("        for (int q = 0; q < 4; ++q) v%d[q] = gx_expr%d(%s[q], %s[q], %s[q]);", o.out, k, a.c_str(), b.c_str(),
            c.c_str());
        else
          t("        for (int q = 0; q < 4; ++q) v%d[q] = point_eval(gop%d, %d, %s, %s[q], %s[q], %s[q]);", o.out, k,
            ov.df, P.vals[o.in[0]].df == DF_F32 ? "true" : "false", a.c_str(), b.c_str(), c.c_str());
      }
      if (L.needs_lds[o.out])
        t("        *(gx_i4*)(L + %s) = gx_i4{v%d[0], v%d[1], v%d[2], v%d[3]};",
          lds_index(o.out, ESV, ESH, "0", "0").c_str(), o.out, o.out, o.out, o.out);
      if (ov.store)
        t("        if (own%s) store4<%s>(%d, (uint8_t*)io.ptr[%d] + (size_t)y * io.pitch[%d], x, W, v%d);",
          edge ? " && y < H" : "", (stream >> o.out) & 1 ? "true" : "false", ov.df, ov.io, ov.io, o.out);
      t("      }");
    }
    t("    }");
  }
};

bool emit_tiles(const GProg& P, int tw_req, int th_req, uint32_t stream, GenSource* out, std::string* why) {
  Layout L;
  plan_stages(P, L);
  int nred = 0;
  for (int k = 0; k < P.nops; ++k) nred += is_reduce_op(P.ops[k].kind) ? 1 : 0;
  const bool red = nred > 0;
  const int hist_words = red ? kGenThreads / 64 * kHistWords : 0;  // a histogram per wave
  static const int shapes[][2] = {{128, 16}, {64, 16}, {64, 8}, {32, 8}, {32, 4}, {16, 4}};
  int TW = 0, TH = 0;
  if (tw_req > 0) {
    if (tw_req % 16 == 0 && th_req > 0 && place_lds(P, L, tw_req, th_req) + hist_words <= kGenLdsBytes / 4) {
      TW = tw_req;
      TH = th_req;
    }
  } else {
    for (auto& s : shapes)
      if (place_lds(P, L, s[0], s[1]) + hist_words <= kGenLdsBytes / 4) {
        TW = s[0];
        TH = s[1];
        break;
      }
  }
  if (!TW) {
    *why = "values kept on chip exceed the LDS budget";
    return false;
  }
  // a tile is interior when every position any stage sweeps, and every
  // input column a window reads, lies inside the image
  int ev_max = 0, eh_max = 0;
  for (int v = 0; v < P.nvals; ++v) {
    ev_max = std::max(ev_max, P.vals[v].ext);
    eh_max = std::max(eh_max, L.eh[v]);
  }
  const int LW = std::max(4, L.lds_words + hist_words);

  Text t;
  bool ok = true;
  emit_prelude(t, P, why, &ok);
  if (!ok) return false;
  t("__device__ constexpr int gx_zero4[4] = {0, 0, 0, 0};");
  // LDS is read and written in whole 16-byte units: consecutive lanes then
  // touch consecutive banks.  A read whose components are not all used would
  // be narrowed to single dwords at a 16-byte lane stride, which hit a
  // quarter of the banks; the empty asm keeps the whole vector.
  t("typedef int gx_i4 __attribute__((ext_vector_type(4)));");
  t("__device__ __forceinline__ gx_i4 gx_ld4(const int32_t* p) {");
  t("  const gx_i4 q = *(const gx_i4*)p;");
  t("  asm volatile(\"\" :: \"v\"(q));");
  t("  return q;");
  t("}");
  // one tile: IN = its halo lies inside the image
  t("template <bool IN>");
  t("__device__ __forceinline__ void gen_tile(const IOTable& io, int W, int H, int tx0, int ty0, int32_t* L%s) {",
    red ? ", RedState& rs" : "");
  bool loads = false;
  for (int v = 0; v < P.nvals; ++v)
    if (P.vals[v].input && L.needs_lds[v]) {
      emit_load(t, P, L, v, TW, TH);
      loads = true;
    }
  if (loads) t("  __syncthreads();");
  int slot_in = 0, slot_edge = 0;
  for (int s = 0; s < L.nstages; ++s) {
    t("  // stage %d: extent %d rows, %d columns", s, L.stage_ev[s], L.stage_eh[s]);
    t("  if constexpr (IN) {");
    StageEmitter{t, P, L, TW, TH, &slot_in, stream}.four_pixels(s, false);
    t("  } else {");
    if (L.resolved) {
      StageEmitter{t, P, L, TW, TH, &slot_edge, stream}.four_pixels(s, true);
      // values of this stage that later windows read: their border
      bool fills = false;
      for (int k = 0; k < P.nops; ++k) {
        const int v = P.ops[k].out;
        if (L.op_stage[k] != s || is_global_op(P.ops[k].kind) || L.bmode[v] < 0) continue;
        if (!fills) t("    __syncthreads();");
        fills = true;
        emit_fill(t, P, L, v, TW, TH);
      }
    } else {
      StageEmitter{t, P, L, TW, TH, &slot_edge, stream}.one_pixel(s);
    }
    t("  }");
    if (s + 1 < L.nstages) t("  __syncthreads();");
  }
  t("}");
  t("extern \"C\" __global__ __launch_bounds__(%d) void hvx_gen(const GProg* __restrict__ P, const IOTable io0,",
    kGenThreads);
  t("                                                           const GenBatchImage* __restrict__ imgs, int nimg,");
  t("                                                           uint32_t* __restrict__ ws) {");
  t("  __shared__ __attribute__((aligned(16))) int32_t L[%d];", LW);
  if (red) {
    t("  RedState rs;");
    t("  red_begin<%d, %d>(rs, (uint32_t*)(L + %d));", kGenThreads, kGenThreads / 64, L.lds_words);
  }
  // Work-groups go to the 8 XCDs in turn (block b to XCD b mod 8), each with
  // its own L2: give every XCD a contiguous run of tiles, so that tiles
  // side by side, whose rows share cache lines, meet in one L2.  A group that
  // reduces takes a contiguous run of tiles of its own.
  t("  const int nb = (int)gridDim.x, b = (int)blockIdx.x;");
  t("  const int per = nb / 8, rem = nb %% 8, xcd = b %% 8;");
  t("  int vb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + b / 8;");
  // one image (the program's size), or one tile of one image of a batch
  t("  IOTable io;");
  t("  int W, H, stride = nb, limit = 1 << 30;");
  t("  if (nimg == 0) {");
  t("    io = io0;");
  t("    W = P->w;");
  t("    H = P->h;");
  t("  } else {");
  t("    const int i = gx_batch_image(imgs, nimg, vb);");
  t("    io = imgs[i].io;");
  t("    W = imgs[i].w;");
  t("    H = imgs[i].h;");
  t("    vb -= imgs[i].block0;");
  t("    limit = vb + 1;  // one tile per work-group");
  t("  }");
  t("  const int tiles_x = (W + %d) / %d;", TW - 1, TW);
  t("  const int ntiles = min(tiles_x * ((H + %d) / %d), limit);", TH - 1, TH);
  t("  const int slot = vb;  // the group's tile, and its slot of partial results when it reduces");
  t("  for (int tile = vb; tile < ntiles; tile += stride) {");
  t("    const int tx0 = (tile %% tiles_x) * %d, ty0 = (tile / tiles_x) * %d;", TW, TH);
  t("    const bool in = tx0 >= %d && ty0 >= %d && tx0 + %d <= W && ty0 + %d <= H;", eh_max, ev_max, TW + eh_max,
    TH + ev_max);
  t("    if (in) gen_tile<true>(io, W, H, tx0, ty0, L%s);", red ? ", rs" : "");
  t("    else gen_tile<false>(io, W, H, tx0, ty0, L%s);", red ? ", rs" : "");
  t("    __syncthreads();  // the tile's LDS is free for the next tile");
  t("  }");
  if (red) t("  red_end_partial<%d>(*P, rs, ws + (size_t)slot * %d);", kGenThreads, red_slot_words(P));
  t("}");
  out->text = t.s;
  out->form = GEN_TILES;
  out->tw = TW;
  out->th = TH;
  out->red = red;
  out->lds_words = LW;
  return true;
}

}  // namespace

// ---- cache, compilation, launch --------------------------------------------------

struct GenKernel {
  int form = 0, tw = 0, th = 0;
  bool red = false;
  int lds_words = 0;
  std::vector<char> code;
  std::mutex mu;
  hipModule_t mod[kMaxDevices] = {};
  hipFunction_t fn[kMaxDevices] = {};
};

namespace {
std::mutex g_cache_mu;
// never freed: code objects stay loaded until the process ends
std::map<std::string, GenKernel*>* g_cache = new std::map<std::string, GenKernel*>();
}  // namespace

bool gen_wanted(const GProg& P) {
  if (P.nops != 1) return true;
  const GOp& o = P.ops[0];
  if (is_global_op(o.kind)) return true;
  if (is_point_op(o.kind)) return o.kind == OP_EXPR;
  // the one-operator local kernel reads a Convolve or NonLinearFilter mask
  // at run time; generated, the mask's zeros and products fold away
  const int in_df = P.vals[o.in[0]].df;
  return o.kind == OP_EXPR_LOCAL || o.kind == OP_CONVOLVE || o.kind == OP_NONLINEAR ||
         (in_df != DF_U8 && in_df != DF_F32);
}

bool gen_source(const GProg& P, int tw, int th, uint32_t stream, GenSource* out, std::string* why) {
  bool any_local = false, any_red = false;
  for (int k = 0; k < P.nops; ++k) {
    const int kind = P.ops[k].kind;
    if (kind == OP_MMLOCS) {
      *why = "the location pass runs alone";
      return false;
    }
    any_local |= is_local(kind);
    any_red |= is_reduce_op(kind);
  }
  if (!any_local && !any_red) return emit_points(P, stream, out, why);
  return emit_tiles(P, tw, th, stream, out, why);
}

const GenKernel* gen_compile(const GenSource& src, std::string* why) {
  std::lock_guard<std::mutex> l(g_cache_mu);
  auto it = g_cache->find(src.text);
  if (it != g_cache->end()) return it->second;
  if (const char* dir = getenv("HVX_GEN_DUMP")) {  // the sources, for reading
    const std::string path = std::string(dir) + "/hvx_gen_" + std::to_string(g_cache->size()) + ".hip";
    if (FILE* f = fopen(path.c_str(), "w")) {
      fputs(src.text.c_str(), f);
      fclose(f);
    }
  }
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.text.c_str(), "hvx_gen.hip", kRtcHeaderCount,
                          const_cast<const char**>(kRtcHeaderTexts),
                          const_cast<const char**>(kRtcHeaderNames)) != HIPRTC_SUCCESS) {
    *why = "hiprtcCreateProgram failed";
    return nullptr;
  }
  const char* opts[] = {"--offload-arch=" HVX_ARCH, "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", "-w"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    *why = std::string("hipRTC: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
    hiprtcDestroyProgram(&prog);
    return nullptr;
  }
  size_t n = 0;
  hiprtcGetCodeSize(prog, &n);
  GenKernel* k = new GenKernel();
  k->code.resize(n);
  hiprtcGetCode(prog, k->code.data());
  hiprtcDestroyProgram(&prog);
  k->form = src.form;
  k->tw = src.tw;
  k->th = src.th;
  k->red = src.red;
  k->lds_words = src.lds_words;
  (*g_cache)[src.text] = k;
  return k;
}

hipError_t gen_load(const GenKernel* kc, int device) {
  GenKernel* k = const_cast<GenKernel*>(kc);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> l(k->mu);
  if (k->fn[device]) return hipSuccess;
  hipModule_t m = nullptr;
  hipError_t e = hipModuleLoadData(&m, k->code.data());
  if (e != hipSuccess) return e;
  hipFunction_t f = nullptr;
  e = hipModuleGetFunction(&f, m, "hvx_gen");
  if (e != hipSuccess) {
    (void)hipModuleUnload(m);
    return e;
  }
  k->mod[device] = m;
  k->fn[device] = f;
  return hipSuccess;
}

hipError_t gen_launch(const GenKernel* k, int device, const GProg& P, const GProg* dev_prog, const IOTable& io,
                      int num_cus, hipStream_t s, uint32_t* ws) {
  if (device < 0 || device >= kMaxDevices || !k->fn[device]) return hipErrorInvalidDeviceFunction;
  long long grid;
  if (k->form == GEN_POINTS) {
    grid = (long long)((P.w + 1023) >> 10) * P.h;
  } else {
    // One work-group per tile (a persistent grid of as many groups as fit
    // the CUs measured slower: the hardware's own dispatch of short groups
    // overlaps one group's loads with another's arithmetic as well).  A
    // group that reduces writes its partial results to its slot of `ws`.
    grid = (long long)((P.w + k->tw - 1) / k->tw) * ((P.h + k->th - 1) / k->th);
    (void)num_cus;
  }
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (k->red && !ws) return hipErrorInvalidValue;
  const GProg* p = dev_prog;
  IOTable t = io;
  const GenBatchImage* none = nullptr;
  int zero = 0;
  void* args[] = {(void*)&p, (void*)&t, (void*)&none, (void*)&zero, (void*)&ws};
  return hipModuleLaunchKernel(k->fn[device], (unsigned)grid, 1, 1, kGenThreads, 1, 1, 0, s, args, nullptr);
}

long long gen_blocks(const GenKernel* k, int w, int h) {
  if (k->form == GEN_POINTS) return (long long)((w + 1023) >> 10) * h;
  return (long long)((w + k->tw - 1) / k->tw) * ((h + k->th - 1) / k->th);
}

bool gen_batchable(const GenKernel* k) { return !k->red; }

hipError_t gen_launch_batch(const GenKernel* k, int device, const GenBatchImage* imgs, int n, long long blocks,
                            hipStream_t s) {
  if (device < 0 || device >= kMaxDevices || !k->fn[device]) return hipErrorInvalidDeviceFunction;
  if (k->red) return hipErrorInvalidValue;
  if (n <= 0 || blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  const GProg* p = nullptr;
  IOTable t;
  memset(&t, 0, sizeof t);
  uint32_t* ws = nullptr;
  void* args[] = {(void*)&p, (void*)&t, (void*)&imgs, (void*)&n, (void*)&ws};
  return hipModuleLaunchKernel(k->fn[device], (unsigned)blocks, 1, 1, kGenThreads, 1, 1, 0, s, args, nullptr);
}

void gen_tile(const GenKernel* k, int* tw, int* th) {
  *tw = k->tw;
  *th = k->th;
}

}  // namespace hvx
