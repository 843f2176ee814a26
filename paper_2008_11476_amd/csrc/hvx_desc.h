// Plain descriptors passed from the host runtime to the kernels by value.
// Shared by host C++ and device code; no HIP types, no pointers to host data.
#pragma once
// hipRTC (kernels generated at run time) provides the HIP and integer types itself
#ifndef __HIPCC_RTC__
#include <stdint.h>
#endif

namespace hvx {

// Point and local operators after lowering (Section 4, Table 2).  Sobel3x3
// lowers to the two local operators SOBEL_X and SOBEL_Y (Section 5.2.2).
enum OpKind : int32_t {
  OP_CHANNEL_Y = 1,
  OP_GAUSS3,
  OP_GAUSS5,
  OP_BOX3,
  OP_BOX5F,
  OP_SOBEL_X,
  OP_SOBEL_Y,
  OP_MAGNITUDE,
  OP_PHASE,
  OP_ADD,
  OP_MULF,
  OP_HARRIS,
  OP_THRESHOLD,
  OP_CONVOLVE,
  OP_DILATE3,  // Table 2 local operators with MAX / MIN / MEDIAN reductions
  OP_ERODE3,
  OP_MEDIAN3,
  OP_NONLINEAR,  // median / min / max over a mask (p0 x p1, p2: 0 median, 1 min, 2 max)
  OP_NONMAX,     // NonMaxSuppression over a (2 p0 + 1)^2 window, U8 or S16
  OP_EXPR,       // user point kernel (Section 5.1): p0 steps of `code`, p1 = 1 float kernel, p2 bit k: input k F32
  OP_EXPR_LOCAL, // user local kernel: as OP_EXPR over one input read at window offsets
  // Global operators (Table 2): each reads every pixel of its input and
  // writes a few values (a buffer, not an image).
  OP_HISTOGRAM,  // U8 -> p0 bins over [p1, p1 + p2), uint32 counts
  OP_MINMAX,     // U8/S16 -> int32 {smallest, largest}
  OP_MMCOUNT,    // U8/S16 -> the extremes and how many pixels equal each (MinMaxLoc counts)
  OP_MMLOCS,     // image, MMCOUNT result -> (x, y) of up to p0 pixels equal to each extreme
  OP_SUMS,       // U8 -> exact sums of v and v^2, mean and standard deviation
  OP_EQHIST,     // U8 -> 256-bin histogram, then the EqualizeHist mapping (a 256-byte table)
  OP_LUT,        // point operator: U8 image, EQHIST table -> U8 (the table applied)
};

// A global operator (its output is a buffer; nothing reads it in the same
// kernel, since it is complete only once every pixel has been seen).
__host__ __device__ inline bool is_global_op(int kind) { return kind >= OP_HISTOGRAM && kind <= OP_EQHIST; }
// A point operator (Section 4): one output pixel from the same pixel of its inputs.
__host__ __device__ inline bool is_point_op(int kind) {
  return kind == OP_CHANNEL_Y || kind == OP_MAGNITUDE || kind == OP_PHASE || kind == OP_THRESHOLD ||
         kind == OP_ADD || kind == OP_MULF || kind == OP_HARRIS || kind == OP_EXPR || kind == OP_LUT;
}
// The global operators a fused kernel can compute as a reduction over its
// tiles (the location lists need the final extremes, so they run apart).
__host__ __device__ inline bool is_reduce_op(int kind) { return is_global_op(kind) && kind != OP_MMLOCS; }

// Bytes of each global operator's result.  EQHIST: the counts, then the
// mapping table.  MMCOUNT: int32 {min, max, count of min, count of max},
// two int32 slot counters of the location lists, two reserved words, then
// the 64-bit (value, count) keys the counting merges into: kMMSubKeys for
// the minimum, kMMSubKeys for the maximum.  Work-group g merges into key
// g mod kMMSubKeys: a compare-and-swap that loses to another group retries
// after a full round trip to the cache, so a key shared by many groups
// serialises them (the streaming kernel has at most kMMSubKeys groups, one
// key each).  The last step merges the keys into the first four words.
constexpr int kEqHistBytes = 256 * 4 + 256;
constexpr int kMinMaxBytes = 8;
constexpr int kMMSubKeys = 256;
constexpr int kMMKeyOffset = 32;  // bytes
constexpr int kMMCountBytes = kMMKeyOffset + 2 * kMMSubKeys * 8;
constexpr int kSumsBytes = 24;

// (value, count) keys of the one-pass count of the extremes: the value in
// the high word, biased by 32768 so that every U8 or S16 value is ordered as
// an unsigned number, the count in the low word.  Merging two keys keeps the
// better value and adds the counts when the values are equal; a key with a
// zero count is neutral, so the minimum starts at (65535, 0) and the maximum
// at (0, 0).
__host__ __device__ inline unsigned long long mm_key(int v, unsigned c) {
  return ((unsigned long long)(unsigned)(v + 32768) << 32) | c;
}
constexpr unsigned long long kMinKeyInit = 0xFFFFull << 32;
constexpr unsigned long long kMaxKeyInit = 0;
__host__ __device__ inline unsigned long long mm_merge(unsigned long long a, unsigned long long b, bool want_min) {
  const unsigned va = (unsigned)(a >> 32), vb = (unsigned)(b >> 32);
  if (va == vb) return a + (unsigned)b;
  return (want_min ? vb < va : vb > va) ? b : a;
}
__host__ __device__ inline int mm_value(unsigned long long k) { return (int)(unsigned)(k >> 32) - 32768; }

// Steps of a user point kernel's postfix program: the low byte is the
// operation, the high byte its argument (input index, literal index).
enum ExprOp : int16_t {
  X_IN = 1, X_CONST, X_ADD, X_SUB, X_MUL, X_DIV, X_NEG, X_MIN, X_MAX, X_ABS, X_CLAMP, X_GT, X_SEL, X_SQRT,
  X_INW  // input a at window offset: argument (dy + 2) * 5 + (dx + 2)
};
constexpr int kMaxExpr = 32;       // steps
constexpr int kMaxExprConst = 8;   // distinct literals
constexpr int kExprStack = 8;      // values on the evaluation stack

// Element formats (same numbering as the public HVX_DF_* constants).
enum Df : int32_t { DF_VIRT = 0, DF_U8 = 1, DF_S16 = 2, DF_S32 = 3, DF_F32 = 4, DF_UYVY = 5,
                   DF_BUF = 16 /* library-internal: a global operator's result, w bytes */ };
enum Border : int32_t { B_UNDEFINED = 0, B_CONSTANT = 1, B_REPLICATE = 2, B_MIRROR = 3, B_REPEAT = 4 };

inline int df_bytes(int df) {
  switch (df) {
    case DF_U8: return 1;
    case DF_S16: return 2;
    case DF_UYVY: return 2;
    case DF_S32: return 4;
    case DF_F32: return 4;
    case DF_BUF: return 1;
    default: return 0;
  }
}

// ---- generic fused-group program (LDS tile interpreter) -------------------
constexpr int kMaxGVals = 16;
constexpr int kMaxGOps = 12;
constexpr int kMaxIO = 8;
constexpr int kMaxMask = 25;
constexpr int kMaxRed = 2;
constexpr int kHistWords = 257;  // 256 bins and a spare counter for pixels outside the range

struct GVal {
  int32_t df;     // element format
  int32_t ext;    // halo (pixels) around the tile over which the value is needed
  int32_t lds;    // offset in 32-bit LDS words of the value's tile, -1 if not kept on chip
  int32_t io;     // index into the I/O table, -1 if the value never touches global memory
  int32_t input;  // 1: read from global memory (a group input)
  int32_t store;  // 1: written to global memory (a group output)
  int32_t wrap;   // 1: a group input whose halo outside the image holds its periodic copies (REPEAT)
};

struct GOp {
  int32_t kind;
  int32_t out;
  int32_t in[3];
  int32_t border;
  int32_t cint;  // border constant for integer inputs
  float cf;      // border constant for F32 inputs
  int32_t rx, ry;
  int32_t p0, p1, p2, p3;  // threshold: true, false, integer bound; add: policy; convolve: cols, rows, shift
  float pf;                // corner response k; threshold bound for F32 input
  int16_t mask[kMaxMask];
  int16_t code[kMaxExpr];      // OP_EXPR program
  int32_t kc[kMaxExprConst];   // OP_EXPR literals (int32, or F32 bits in a float kernel)
};

struct GProg {
  int32_t nvals, nops;
  int32_t tw, th;     // output tile of one work-group
  int32_t lds_words;  // LDS words used by one tile (a histogram, if any, follows: kHistWords)
  int32_t nred;       // global operators reduced over the tiles (at most kMaxRed, one histogram)
  int32_t w, h;
  int32_t tiles_x, tiles_y;
  GVal vals[kMaxGVals];
  GOp ops[kMaxGOps];
};

struct IOTable {
  void* ptr[kMaxIO];
  int64_t pitch[kMaxIO];
};

// ---- fast fused kernels -------------------------------------------------------
// Work decomposition shared by the register-streaming kernels: a wave owns a
// vertical strip of 60 * 16 output columns (plus one halo lane on each side)
// and a band of `rows` output rows, streamed top to bottom.  960 columns keep
// every strip's rows 64-byte aligned; misaligned 992-column strips streamed
// about 15% slower on the HBM.
constexpr int kLanePx = 16;
constexpr int kOutLanes = 60;
constexpr int kStripPx = kOutLanes * kLanePx;

struct StripGrid {
  int32_t w, h;
  int32_t rows;     // output rows per work item
  int32_t nstrips;  // ceil(w / kStripPx)
  int32_t nbands;   // ceil(h / rows)
};

// Gaussian3x3 -> Sobel3x3 -> Magnitude -> Threshold (and optionally Phase).
struct EdgeDesc {
  StripGrid g;
  const uint8_t* in;
  int64_t in_pitch;
  uint8_t* out;  // threshold output
  int64_t out_pitch;
  uint8_t* phase;  // phase output or null
  int64_t phase_pitch;
  int32_t b0, c0;   // border of the Gaussian's input
  int32_t b1, c1;   // border of the Sobel's input
  int32_t thr_not;  // edge iff gx^2 + gy^2 + thr_not >= 0 (thr_not = ~T, T = u(u-1))
  uint32_t tv4, fv4;
};

// Sobel3x3 -> products -> Box5x5 (x3) -> corner response -> Threshold.
struct CornerDesc {
  StripGrid g;
  const uint8_t* in;
  int64_t in_pitch;
  uint8_t* out;
  int64_t out_pitch;
  int32_t b0, c0;  // border of the Sobel's input
  int32_t b1;      // border of the box filters' inputs
  float c1;        // their constant
  float k;
  float thr;  // response threshold (strict >), as the largest float not above the value
  uint32_t tv4, fv4;
};

// Gaussian5x5, optionally fed by the luma of a UYVY frame.
struct Gauss5Desc {
  StripGrid g;
  const uint8_t* in;
  int64_t in_pitch;
  int32_t uyvy;  // 1: input is UYVY, take its luma
  uint8_t* out;
  int64_t out_pitch;
  int32_t b0, c0;
};

// FK_GLOBAL: one global operator over an image in memory (the streaming
// reduction kernels of the immediate-mode calls).
enum FastKind : int32_t { FK_GENERIC = 0, FK_EDGE = 1, FK_CORNER = 2, FK_GAUSS5 = 3, FK_GLOBAL = 4 };
// the register-streaming strip kernels (work items of strips x bands; batchable)
inline bool is_strip_kind(int k) { return k == FK_EDGE || k == FK_CORNER || k == FK_GAUSS5; }

// One image of a batch: the kind selects which fused body processes its items.
struct BatchImage {
  int32_t kind;
  int32_t first_item;  // index of its first work item in the flat work list
  int32_t nitems;
  int32_t pad;
  union {
    EdgeDesc e;
    CornerDesc c;
    Gauss5Desc g5;
  } d;
};

}  // namespace hvx
