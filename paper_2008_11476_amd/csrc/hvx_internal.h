// Host-side objects, graph IR and launch plan of the hvx library.
#pragma once
#include <stdint.h>

#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hvx.h"
#include "expr.h"
#include "hvx_desc.h"

namespace hvx {

enum ObjType : uint32_t { T_CONTEXT = 0x5a01, T_GRAPH, T_IMAGE, T_NODE, T_CONV, T_BATCH, T_SERVER, T_BUFFER };

struct Context;
struct Graph;
struct GenKernel;  // codegen.h
struct TuneEntry;

struct Object {
  uint32_t type;
  Context* ctx;
  virtual ~Object() {}
};

// An image, or (type T_BUFFER) a caller's device buffer receiving a global
// operator's result: df DF_BUF, w = its size in bytes, h = 1.
struct Image : Object {
  uint32_t w = 0, h = 0;
  int df = DF_VIRT;
  bool is_virtual = false;
  Graph* vgraph = nullptr;  // owning graph of a virtual image
  void* ptr = nullptr;
  size_t pitch = 0;
  bool owned = false;  // device memory allocated by the library
};

struct Conv : Object {
  uint32_t cols = 0, rows = 0, scale = 1;
  std::vector<int16_t> coeffs;
};

// OpenVX function nodes as the user adds them.
enum NodeKind : int32_t {
  NK_CHANNEL_EXTRACT = 1,
  NK_GAUSS3,
  NK_GAUSS5,
  NK_BOX3,
  NK_DILATE3,
  NK_ERODE3,
  NK_MEDIAN3,
  NK_NONLINEAR,
  NK_NONMAX,
  NK_BOX5F,
  NK_SOBEL3,
  NK_MAGNITUDE,
  NK_PHASE,
  NK_ADD,
  NK_MULF,
  NK_HARRIS,
  NK_THRESHOLD,
  NK_CONVOLVE,
  NK_CUSTOM_POINT,
  NK_CUSTOM_LOCAL,
  NK_HISTOGRAM,  // global operators (Table 2)
  NK_MINMAX,
  NK_MINMAXLOC,
  NK_MEANSTD,
  NK_EQHIST,
};

struct Node : Object {
  Graph* g = nullptr;
  int kind = 0;
  std::vector<Image*> in;   // inputs in API order
  std::vector<Image*> out;  // outputs in API order (may hold nulls: Sobel)
  int border = B_REPLICATE;
  uint32_t bconst = 0;
  double dval = 0;  // threshold value
  int tv = 255, fv = 0;
  int policy = 0;
  float k = 0.04f;
  Conv* conv = nullptr;
  int channel = 0;
  Conv own_mask;  // NonLinearFilter: the node's own copy of its mask (conv points here)
  ExprProg expr;  // user point kernel
  int out_df = 0; // user point kernel: declared output format
  uint32_t gp[3] = {0, 0, 0};  // histogram: bins, offset, range; MinMaxLoc: location capacity
};

// ---- lowered graph and plan -------------------------------------------------

struct Value {
  Image* img = nullptr;
  int df = DF_VIRT;
  uint32_t w = 0, h = 0;
  bool is_virtual = false;
  int producer = -1;           // lowered op writing it, -1 for graph inputs
  std::vector<int> consumers;  // lowered ops reading it (live ones after DCE)
  bool live = false;
  // materialised device copy (virtual values crossing kernel boundaries)
  bool materialize = false;
};

struct LOp {
  int kind = 0;
  int node = -1;  // index of the function node it came from
  int in[3] = {-1, -1, -1};
  int nin = 0;
  int out = -1;
  int border = B_REPLICATE;
  uint32_t bconst = 0;
  double dval = 0;
  int tv = 255, fv = 0, policy = 0;
  float k = 0.04f;
  const Conv* conv = nullptr;
  const ExprProg* expr = nullptr;
  uint32_t gp[3] = {0, 0, 0};  // global operators: as Node::gp
  int rx = 0, ry = 0;
  bool live = true;
};

struct Group {
  std::vector<int> ops;      // lowered ops, topological order
  std::vector<int> inputs;   // values read from global memory
  std::vector<int> outputs;  // values written to global memory
  std::vector<int> gvals;    // generic program value index -> plan value id
  int kind = FK_GENERIC;
  int phase = 0;             // global operators whose results this group waits for (launch order)
  int footprint = 0;  // max total stencil radius along any path
  GProg prog{};       // generic program (kind == FK_GENERIC)
  const GenKernel* gen = nullptr;  // kernel generated for `prog` (null: the tile interpreter)
  int rows = 0;       // rows per work item (fast kinds); 0 = tuned or default
  int xcd = 1;        // XCD-contiguous work mapping
  uint32_t w = 0, h = 0;
  // indices (into Plan::vals) bound to the fast descriptors' pointers
  int v_in = -1, v_out = -1, v_aux = -1;
};

struct Plan {
  std::vector<Value> vals;
  std::vector<LOp> ops;
  std::vector<Group> groups;
  int num_nodes = 0, num_ops = 0, num_live = 0;
  int64_t alg_bytes = 0, hbm_bytes = 0, scratch_bytes = 0;
  int num_generated = 0;  // groups run by generated kernels
  std::string op_key;     // operator signature: the tune-cache key of plan choices
  std::vector<int> cuts;  // values at which fusion was cut (plan choice)
  std::vector<std::array<int, 3>> tiles;  // tiles of generated groups (plan choice)
  std::string gen_note;   // why a group was left to the interpreter (last case)
  std::vector<int> topo;  // live op order
};

struct Graph : Object {
  std::vector<Node*> nodes;
  std::vector<Image*> virt;
  bool verified = false;
  int opt_fusion = 1, opt_dce = 1, opt_tile = 0, opt_specialize = 1, opt_xcd = 1, opt_codegen = 1;
  // plan choice in force for the next verification (set by the tuner while
  // it times candidates); null: the tune cache's choice for the graph, if any
  const TuneEntry* plan_choice = nullptr;
  std::unique_ptr<Plan> plan;
  // device state: the materialised values live in one block of scratch_total
  // bytes, value v at scratch_off[v] with row pitch scratch_pitch[v] (0: not
  // materialised); a served request runs the plan on a block of its own
  char* scratch_base = nullptr;
  size_t scratch_total = 0;
  bool prepared = false;
  std::vector<size_t> scratch_off;
  std::vector<size_t> scratch_pitch;
  std::vector<size_t> ws_off;  // per group: workspace of a generated reducing kernel in the scratch block
  GProg* dev_progs = nullptr;  // device copies of the groups' generic programs (index = group)
  void* last_stream = nullptr;
  bool scheduled = false;
};

struct TuneEntry {
  int rows = 0;
  int xcd = 1;
  double us = 0;
  // a plan choice (key "plan|" + the operator signature): the values at
  // which fusion is cut and the tiles of generated groups (first operator,
  // width, height)
  bool has_plan = false;
  std::vector<int> cuts;
  std::vector<std::array<int, 3>> tiles;
};

struct Context : Object {
  int device = 0;
  std::recursive_mutex mu;
  std::string last_error;
  std::vector<Object*> children;  // every object created in this context
  bool dev_ready = false;
  int num_cus = 256;
  std::string dev_name;
  std::map<std::string, TuneEntry> tune;  // key: device|signature|size
};

// ---- registry and errors ----------------------------------------------------
bool registry_check(const void* h, uint32_t type);
void registry_add(Object* o);
void registry_remove(Object* o);
hvx_status set_error(Context* ctx, hvx_status s, const char* fmt, ...);

// ---- planner (verify.cpp) ---------------------------------------------------
hvx_status verify_graph(Graph* g);
std::string graph_signature(const Graph* g);

// ---- runtime (runtime.cpp) --------------------------------------------------
// Device memory of one execution of a plan in place of the graph's own: the
// non-virtual values listed in `ptr` (index = value id; null = the image's
// own pointer) and a scratch block for the materialised values (null = the
// graph's).  Used by the server to run a template on a request's buffers.
struct Bind {
  std::vector<void*> ptr;
  std::vector<int64_t> pitch;
  char* scratch = nullptr;
};
hvx_status ensure_device(Context* ctx);
hvx_status prepare_graph(Graph* g);
hvx_status schedule_graph(Graph* g, void* stream);
hvx_status schedule_bound(Graph* g, void* stream, const Bind* b);
void free_graph_device(Graph* g);
int default_rows(const Group& gr, int num_cus);
int rows_for(const Graph* g, const Group& gr);  // rows per work item in effect (option, tuned, default)
void fill_fast_desc(const Graph* g, const Group& gr, BatchImage* bi, int rows_override = 0, const Bind* b = nullptr);
int64_t fast_items(const Group& gr);

}  // namespace hvx
