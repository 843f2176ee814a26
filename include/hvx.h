/*
 * hvx: OpenVX-style image graphs executed as fused HIP kernels on gfx950.
 *
 * The calls follow the graph formulation of OpenVX as the paper uses it
 * (Section 3.1 and its edge-detection listing): create a context and a graph,
 * create images (some of them virtual), add function nodes, verify the graph,
 * then process it, possibly many times with new frames.  Verification is
 * where the graph is checked and optimised (Section 5.2): parameter checks,
 * cycle and bipartiteness checks, lowering of each node to point and local
 * operators (Section 4, Table 2), elimination of dead computations
 * (Section 5.2.2, Algorithm 1), fusion of producer/consumer operators so that
 * intermediates stay on chip (Section 6.3), and the launch plan.
 *
 * Conventions (apply to every call):
 *  - Every call returns an hvx_status; no C++ exception crosses this
 *    boundary.  Handles are checked against a registry: a released or
 *    foreign handle gives HVX_ERROR_INVALID_REFERENCE, never a crash.
 *  - hvx_last_error(ctx) returns a message for the context's last failure.
 *  - Device pointers passed in (hvx_image_from_ptr, hvx_image_swap_ptr) are
 *    BORROWED: the library never frees them, and the caller keeps them alive
 *    until the work that uses them has completed (hvx_graph_wait, or a
 *    synchronisation of the stream given to hvx_graph_schedule).
 *  - Images made by hvx_image_create and virtual images are owned by the
 *    library and freed when released, or when their context is released.
 *  - Pixel layout: row-major, row y starts at byte y * pitch.  The pitch of
 *    every device image must be a multiple of 64 bytes and at least
 *    width * bytes-per-pixel.  Bytes between the end of a row and the next
 *    pitch boundary are padding: the library may read them, and kernels may
 *    overwrite the padding of OUTPUT images; pixel data is never touched
 *    outside the images a node writes.
 *  - Not thread-safe per graph: calls on one graph must not overlap.
 *    Distinct graphs and servers may be used from distinct threads.
 */
#ifndef HVX_H
#define HVX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hvx_context_s* hvx_context;
typedef struct hvx_graph_s* hvx_graph;
typedef struct hvx_image_s* hvx_image;
typedef struct hvx_node_s* hvx_node;
typedef struct hvx_conv_s* hvx_convolution;
typedef struct hvx_batch_s* hvx_batch;
typedef struct hvx_server_s* hvx_server;
typedef struct hvx_buffer_s* hvx_buffer;

typedef int32_t hvx_status;
#define HVX_SUCCESS 0
#define HVX_ERROR_INVALID_REFERENCE (-1)  /* null, released or wrong-type handle */
#define HVX_ERROR_INVALID_PARAMETERS (-2) /* bad value of a scalar argument */
#define HVX_ERROR_INVALID_FORMAT (-3)     /* image format not accepted by the node */
#define HVX_ERROR_INVALID_DIMENSION (-4)  /* image sizes do not match */
#define HVX_ERROR_INVALID_GRAPH (-5)      /* cycle, not bipartite, two writers, foreign image */
#define HVX_ERROR_NOT_VERIFIED (-6)       /* graph changed or never verified */
#define HVX_ERROR_NO_MEMORY (-7)          /* host/device allocation or HBM budget */
#define HVX_ERROR_NOT_SUPPORTED (-8)
#define HVX_ERROR_DEVICE (-9)             /* a HIP call failed or no device is present */

/* Image formats.  Bytes per pixel: U8 1, S16 2, S32 4, F32 4, UYVY 2. */
#define HVX_DF_VIRT 0 /* only for virtual images: resolved at verification */
#define HVX_DF_U8 1
#define HVX_DF_S16 2
#define HVX_DF_S32 3
#define HVX_DF_F32 4
#define HVX_DF_UYVY 5 /* 4:2:2, bytes U Y0 V Y1 per pixel pair; width must be even */

/* Border modes of a local operator's input (applied per node). */
#define HVX_BORDER_UNDEFINED 0 /* output pixels whose window leaves the image are unspecified */
#define HVX_BORDER_CONSTANT 1  /* pixels outside the image read as the constant */
#define HVX_BORDER_REPLICATE 2 /* pixels outside the image read as the nearest edge pixel */
#define HVX_BORDER_MIRROR 3    /* the image reflected about its first and last pixel (reflect-101),
                                  repeated; a one-pixel axis repeats its pixel.  Graphs using it
                                  run on the generic kernels. */
#define HVX_BORDER_REPEAT 4    /* the image tiled periodically: position x reads x mod width (same
                                  for rows).  Graphs using it run on the generic kernels, and a
                                  fused group in which such a node reads an intermediate of the
                                  group runs node by node instead. */

#define HVX_POLICY_SATURATE 0
#define HVX_POLICY_WRAP 1

#define HVX_CHANNEL_Y 0

/* Graph options (hvx_graph_set_option).  Changing one un-verifies the graph. */
#define HVX_OPT_FUSION 1     /* 1 (default): fuse producer/consumer operators; 0: one kernel per operator */
#define HVX_OPT_DCE 2        /* 1 (default): remove operators whose results reach no non-virtual image */
#define HVX_OPT_TILE 3       /* 0 (default): tuned/default tiles; else rows per work item (fast kernels) */
#define HVX_OPT_SPECIALIZE 4 /* 1 (default): use hand-fused kernels for recognised subgraphs; 0: generic */
#define HVX_OPT_XCD_REMAP 5  /* 1 (default): map work items to XCDs in contiguous chunks */
#define HVX_OPT_CODEGEN 6    /* 1 (default): a kernel generated and compiled (hipRTC) per fused group that
                                has no hand-fused kernel (Section 6); 0: the tile interpreter runs it.
                                Environment: HVX_GEN_LOG set prints why a group was left to the
                                interpreter; HVX_GEN_DUMP=<dir> writes each generated source there */

/* Graph queries (hvx_graph_query); valid after verification. */
#define HVX_QUERY_NUM_NODES 1      /* function nodes added */
#define HVX_QUERY_NUM_OPS 2        /* point/local operators after lowering */
#define HVX_QUERY_NUM_LIVE_OPS 3   /* operators left after dead-computation elimination */
#define HVX_QUERY_NUM_KERNELS 4    /* fused kernels per process call (not counting the one-group steps that
                                      start and finish a global operator's result) */
#define HVX_QUERY_ALG_BYTES 5      /* bytes a process call must move: inputs read once, outputs written once */
#define HVX_QUERY_HBM_BYTES 6      /* bytes the plan moves, materialised intermediates included (no halos) */
#define HVX_QUERY_KERNEL_KIND 7    /* kind of the first kernel: 0 generic, 1 edge, 2 corner, 3 gauss5,
                                      4 one global operator */
#define HVX_QUERY_SCRATCH_BYTES 8  /* device bytes of materialised intermediates */
#define HVX_QUERY_OP_LIVE_MASK 9   /* bit i set: lowered operator i is live (first 63 operators) */
#define HVX_QUERY_ROWS_PER_ITEM 10 /* rows per work item of the first kernel */
#define HVX_QUERY_NUM_GENERATED 11 /* kernels of the plan generated for their group (HVX_OPT_CODEGEN) */
#define HVX_QUERY_PLAN_CUTS 12     /* values at which the plan choice in force cuts fusion */
#define HVX_QUERY_GEN_TILE 13      /* tile of the first generated tile kernel: width << 16 | height (0: none) */

/* ---- context ------------------------------------------------------------ */

/* Create a context bound to HIP device `hip_device`.  No device work happens
 * until something needs the device, so graphs can be built and verified on a
 * machine without a GPU.  Context (Section 3.1). */
hvx_status hvx_context_create(int hip_device, hvx_context* out);
/* Release a context and every object created in it (images, graphs, nodes,
 * convolutions, batches, servers); waits for their device work first.
 * *ctx is set to NULL.  Implicit freeing at context release (Section 3.1). */
hvx_status hvx_context_release(hvx_context* ctx);
/* Message for the last failed call made with this context (never NULL). */
const char* hvx_last_error(hvx_context ctx);
/* Name of a status code (never NULL). */
const char* hvx_status_name(hvx_status s);

/* ---- images ------------------------------------------------------------- */

/* Wrap caller-owned device memory (w x h pixels of format df, row pitch in
 * bytes).  Non-virtual images are the data a program can read and write
 * (Section 5.2.1). */
hvx_status hvx_image_from_ptr(hvx_context ctx, uint32_t w, uint32_t h, int df, void* dev_ptr, size_t pitch_bytes,
                              hvx_image* out);
/* Allocate a device image owned by the library (pitch rounded up to 64). */
hvx_status hvx_image_create(hvx_context ctx, uint32_t w, uint32_t h, int df, hvx_image* out);
/* Point a non-virtual image at a new frame of the same size and format; a
 * verified graph stays verified (a verified graph runs repeatedly on new
 * frames, Section 3.1). */
hvx_status hvx_image_swap_ptr(hvx_image img, void* dev_ptr, size_t pitch_bytes);
/* Describe an image: any output pointer may be NULL. */
hvx_status hvx_image_query(hvx_image img, uint32_t* w, uint32_t* h, int* df, void** dev_ptr, size_t* pitch_bytes);
/* Copy between host memory (row pitch host_pitch bytes) and a non-virtual
 * image; synchronous.  to_device = 1 writes the image, 0 reads it. */
hvx_status hvx_image_copy(hvx_image img, void* host, size_t host_pitch, int to_device);
/* An intermediate image of one graph: not host-accessible; w, h = 0 and
 * df = HVX_DF_VIRT mean "inferred at verification" (Section 3.1). */
hvx_status hvx_image_create_virtual(hvx_graph graph, uint32_t w, uint32_t h, int df, hvx_image* out);

/* Integer convolution mask: cols x rows coefficients (odd sizes 1..5),
 * row-major, centre at (cols/2, rows/2); scale must be a power of two
 * (1..2^15).  Copied. */
hvx_status hvx_convolution_create(hvx_context ctx, uint32_t cols, uint32_t rows, const int16_t* coeffs,
                                  uint32_t scale, hvx_convolution* out);

/* Wrap caller-owned device memory of `bytes` bytes (8-byte aligned) that a
 * global operator node writes its result into: a global operator reads every
 * pixel of an image and produces a few values rather than an image (Table 2).
 * BORROWED like hvx_image_from_ptr.  A buffer is a non-virtual data object
 * of the graph: the node writing it is never dead code.  Verification checks
 * that it is large enough (INVALID_DIMENSION).  INVALID_PARAMETERS for a
 * NULL or misaligned pointer, INVALID_DIMENSION for 0 or more than 2^31
 * bytes. */
hvx_status hvx_buffer_from_ptr(hvx_context ctx, void* dev_ptr, size_t bytes, hvx_buffer* out);

/* ---- graph and nodes ---------------------------------------------------- */

/* An empty graph in `ctx` (the graph object of Section 3.1).
 * INVALID_REFERENCE for a bad context, INVALID_PARAMETERS for a NULL out. */
hvx_status hvx_graph_create(hvx_context ctx, hvx_graph* out);

/* Node constructors.  Each adds one OpenVX function node to the graph and
 * un-verifies it; `node_out` may be NULL.  Inputs precede outputs.  Formats
 * are checked at verification.  The arithmetic of each node:
 *  channel_extract  UYVY -> U8: the luma byte of each pixel.
 *  gaussian3x3      U8 -> U8: sum of (1 2 1)x(1 2 1)-weighted window, >> 4.
 *  gaussian5x5      U8 -> U8: sum of (1 4 6 4 1)^2-weighted window, >> 8.
 *  box3x3           U8 -> U8: window sum / 9, floor.
 *  dilate3x3        U8 -> U8: largest pixel of the 3x3 window.
 *  erode3x3         U8 -> U8: smallest pixel of the 3x3 window.
 *  median3x3        U8 -> U8: median (fifth smallest) of the 3x3 window.
 *  nonlinear_filter U8 -> U8: median, minimum or maximum of the window pixels
 *                   selected by a mask; the median of n pixels is the one at
 *                   index n / 2 of their ascending order.
 *  box5x5_f32       F32 -> F32: unnormalised 5x5 window sum.
 *  sobel3x3         U8 -> S16 gx (right minus left), S16 gy (bottom minus top),
 *                   (1 2 1) smoothing across; either output may be NULL.
 *  magnitude        S16,S16 -> S16: sqrt(gx^2+gy^2) rounded half up (no ties occur
 *                   for integer sums), saturated to 32767.
 *  phase            S16,S16 -> U8: atan2(gy,gx) in [0,2pi) scaled to 256 levels,
 *                   rounded, modulo 256 (within 1 level of the exact value).
 *  add              U8/S16 -> U8/S16 with HVX_POLICY_SATURATE or _WRAP.
 *  multiply_f32     S16,S16 -> F32: exact product (custom point node).
 *  harris_response  F32 x3 (Sxx, Syy, Sxy) -> F32: Sxx*Syy - Sxy^2 - k (Sxx+Syy)^2
 *                   (custom point node).
 *  threshold        U8/S16/F32 -> U8: true_v where in > value, else false_v.
 *  convolve         U8 -> U8/S16: true convolution with the mask, / scale
 *                   truncated toward zero, saturated.
 * Point and local operators as in Section 4 and Table 2; Sobel is lowered to
 * two local operators (Section 5.2.2). */
hvx_status hvx_channel_extract_node(hvx_graph g, hvx_image uyvy, int channel, hvx_image out, hvx_node* node_out);
hvx_status hvx_gaussian3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);
hvx_status hvx_gaussian5x5_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);
hvx_status hvx_box3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);
/* Table 2 local operators with a MAX / MIN / MEDIAN reduction over the window */
hvx_status hvx_dilate3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);
hvx_status hvx_erode3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);
hvx_status hvx_median3x3_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);
hvx_status hvx_box5x5_f32_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);
hvx_status hvx_sobel3x3_node(hvx_graph g, hvx_image in, hvx_image gx, hvx_image gy, hvx_node* node_out);
hvx_status hvx_magnitude_node(hvx_graph g, hvx_image gx, hvx_image gy, hvx_image out, hvx_node* node_out);
hvx_status hvx_phase_node(hvx_graph g, hvx_image gx, hvx_image gy, hvx_image out, hvx_node* node_out);
hvx_status hvx_add_node(hvx_graph g, hvx_image a, hvx_image b, int policy, hvx_image out, hvx_node* node_out);
hvx_status hvx_multiply_f32_node(hvx_graph g, hvx_image a, hvx_image b, hvx_image out, hvx_node* node_out);
hvx_status hvx_harris_response_node(hvx_graph g, hvx_image sxx, hvx_image syy, hvx_image sxy, float k,
                                    hvx_image out, hvx_node* node_out);
hvx_status hvx_threshold_node(hvx_graph g, hvx_image in, double value, uint8_t true_v, uint8_t false_v,
                              hvx_image out, hvx_node* node_out);
hvx_status hvx_convolve_node(hvx_graph g, hvx_image in, hvx_convolution conv, hvx_image out, hvx_node* node_out);
/* NonLinearFilter (Table 2 local operator).  `mask` is cols x rows bytes,
 * row-major, centred on the output pixel (odd sizes up to 5x5, at least one
 * nonzero entry: INVALID_DIMENSION / INVALID_PARAMETERS otherwise); nonzero
 * entries select window pixels.  The mask is copied. */
#define HVX_NONLINEAR_MEDIAN 0
#define HVX_NONLINEAR_MIN 1
#define HVX_NONLINEAR_MAX 2
hvx_status hvx_nonlinear_filter_node(hvx_graph g, int function, hvx_image in, uint32_t cols, uint32_t rows,
                                     const uint8_t* mask, hvx_image out, hvx_node* node_out);
/* NonMaxSuppression (Table 2 local operator), U8 -> U8 or S16 -> S16 over a
 * win_size x win_size window (3 or 5; INVALID_PARAMETERS otherwise).  A pixel
 * is kept where every window pixel before it in raster order is smaller and
 * every one after it is not larger; elsewhere the output is the format's
 * minimum (0, -32768).  Of a plateau of equal maxima only the first pixel in
 * raster order survives.  Window positions outside the image are read
 * through the node's border mode, and a border copy of the pixel itself
 * counts like any other position (so under REPLICATE row 0 and column 0 are
 * always suppressed). */
hvx_status hvx_non_max_suppression_node(hvx_graph g, hvx_image in, uint32_t win_size, hvx_image out,
                                        hvx_node* node_out);

/* User-defined point kernel (Section 5.1): `expr` computes each output pixel
 * from the pixels at the same position of 1 to 3 inputs, named a, b, c.  It
 * is parsed once here (INVALID_PARAMETERS with the position of the error
 * otherwise), and the node is analysed, dead-code eliminated and fused like
 * the built-in point operators.  Grammar: integer or decimal literals, a / b
 * / c, unary -, binary + - * / with the usual precedence, parentheses, and
 * min(x, y), max(x, y), abs(x), clamp(x, lo, hi) = min(max(x, lo), hi),
 * gt(x, y) (1 where x > y, else 0), sel(p, x, y) (x where p != 0, else y),
 * sqrt(x).  At most 32 steps (names, literals and operations), 8 distinct
 * literals and 8 values pending at once.
 *   Integer kernel (every input U8/S16, out_format U8 or S16): 32-bit two's
 *   complement arithmetic; + - * and negation wrap modulo 2^32, / truncates
 *   toward zero, x / 0 = 0, (-2^31) / (-1) = -2^31; the result saturates to
 *   the output format.  Literals are integers that fit 32 bits; no sqrt.
 *   Float kernel (an F32 input or out_format F32; the output must be F32):
 *   F32 arithmetic with IEEE division and square root.
 * Format errors are reported by verification (INVALID_FORMAT).  `inputs` is
 * read during the call only. */
hvx_status hvx_custom_point_node(hvx_graph g, const char* expr, const hvx_image* inputs, uint32_t num_inputs,
                                 int out_format, hvx_image out, hvx_node* node_out);

/* Global operators (Table 2), immediate mode: each call reads the whole
 * (non-virtual) image and writes its result to caller-owned device memory,
 * asynchronously on `stream` (NULL: the default stream); the image and the
 * buffer must stay valid until the stream reaches the call.  The result is
 * initialised by a kernel in the same stream, so the calls can be captured
 * into a HIP graph.  Calls that share a result buffer and overlap race.
 * INVALID_REFERENCE / INVALID_FORMAT / INVALID_PARAMETERS as stated; DEVICE
 * if a launch fails.
 *  histogram: U8 image; dev_counts holds num_bins uint32 counts.  A pixel v
 *    with offset <= v < offset + range falls in bin (v - offset) * num_bins /
 *    range (integer division); other pixels are not counted.  Needs
 *    1 <= num_bins <= range and offset + range <= 256.
 *  min_max: U8 or S16 image; dev_min_max receives {smallest, largest}.
 *  min_max_count: U8 or S16 image; dev_result (4128 bytes, 8-byte aligned)
 *    receives {smallest, largest, number of pixels equal to the smallest,
 *    number equal to the largest} (the counts of MinMaxLoc) in its first 4
 *    int32, all from one pass over the image; the call uses the rest while
 *    counting.
 *  min_max_loc: as min_max_count, and the (x, y) of the pixels equal to
 *    each extreme, two uint32 per location, into dev_min_locs / dev_max_locs
 *    (capacity locations each; both may be NULL when capacity is 0), from a
 *    second pass that stops once both lists are full.  dev_result (4128
 *    bytes, 8-byte aligned): the 4 results, then 2 int32 the call uses as
 *    slot counters (reservations; min(counter, capacity) locations are
 *    stored), then words used while counting.  When
 *    an extreme occurs more than capacity times, capacity of its locations
 *    are kept; which ones, and the order of any list, are unspecified.
 *  equalize_hist: U8 image -> U8 image `out` of the same size (may be the
 *    input).  With cdf(v) the pixels <= v, cdf_min the smallest nonzero
 *    cdf and N the pixel count, v maps to round((cdf(v) - cdf_min) * 255 /
 *    (N - cdf_min)), halves up; an image of one value is copied unchanged.
 *    dev_workspace: 1280 bytes of device memory, 4-byte aligned (the
 *    histogram and the mapping), used until the stream reaches the call.
 *  mean_std_dev: U8 image; dev_result (24 bytes, 8-byte aligned) receives
 *    the exact sums uint64 S1 = sum v and S2 = sum v^2, then float mean =
 *    S1 / N and float population standard deviation sqrt(S2 / N - mean^2),
 *    both formed in double precision. */
hvx_status hvx_histogram(hvx_context ctx, hvx_image in, uint32_t num_bins, uint32_t offset, uint32_t range,
                         uint32_t* dev_counts, void* stream);
hvx_status hvx_min_max(hvx_context ctx, hvx_image in, int32_t* dev_min_max, void* stream);
hvx_status hvx_min_max_count(hvx_context ctx, hvx_image in, int32_t* dev_result, void* stream);
hvx_status hvx_min_max_loc(hvx_context ctx, hvx_image in, int32_t* dev_result, uint32_t* dev_min_locs,
                           uint32_t* dev_max_locs, uint32_t capacity, void* stream);
hvx_status hvx_equalize_hist(hvx_context ctx, hvx_image in, hvx_image out, void* dev_workspace, void* stream);
hvx_status hvx_mean_std_dev(hvx_context ctx, hvx_image in, void* dev_result, void* stream);

/* EqualizeHist for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * hvx_equalize_hist with the same arguments, arithmetic and errors, minus
 * the workspace.  The 1280 bytes of histogram and mapping come from a fixed
 * device array inside the library, one per GPU, held until the process
 * ends; the call allocates nothing (no hipMalloc, no allocating library
 * routine).  Limit: images of fewer than 2^31 pixels (INVALID_DIMENSION
 * otherwise), as for every global operator.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (on different streams, or
 * from different threads) race and give undefined results; calls ordered on
 * one stream are safe, since each call clears what it counts in a kernel of
 * its own stream.  DEVICE if the array's address cannot be resolved or a
 * launch fails. */
hvx_status hvx_equalize_hist_noalloc(hvx_context ctx, hvx_image in, hvx_image out, void* stream);

/* Global operator nodes (Table 2), the graph form of the immediate-mode
 * calls above: verified, ordered and dead-code eliminated with the rest of
 * the graph.  A point or local producer of the node's input is fused into the
 * reduction (one kernel computes the producer over its tiles and reduces its
 * values without writing them to memory).  Anything that reads a global
 * operator's result runs in a later kernel, since the result is complete
 * only once every pixel has been counted.  Results, byte layouts:
 *  histogram_node: U8 image; `counts` num_bins uint32 (bins as in
 *    hvx_histogram; INVALID_PARAMETERS for bad bins/offset/range).
 *  min_max_node: U8 or S16 image; `result` 2 int32 {smallest, largest}.
 *  min_max_loc_node: U8 or S16 image; `result` 4128 bytes: 8 int32
 *    {smallest, largest, pixels equal to the smallest, pixels equal to the
 *    largest, locations stored in each of the two lists (at most capacity; 0
 *    without locations), 2 reserved}, then 4096 bytes used while counting;
 *    `locations` (NULL exactly when capacity is 0) 4 * capacity uint32: up
 *    to capacity (x, y) pairs of pixels equal to the smallest value, then
 *    capacity pairs for the largest; which ones are kept when an extreme
 *    occurs more often, and their order, are unspecified.  The locations take
 *    a second pass over the image (materialised if it is virtual).
 *  mean_std_dev_node: U8 image; `result` 24 bytes as in hvx_mean_std_dev.
 *  equalize_hist_node: U8 image -> U8 image of the same size (a point
 *    operator applying the mapping of hvx_equalize_hist; the histogram and
 *    mapping live in the graph's device memory). */
hvx_status hvx_histogram_node(hvx_graph g, hvx_image in, uint32_t num_bins, uint32_t offset, uint32_t range,
                              hvx_buffer counts, hvx_node* node_out);
hvx_status hvx_min_max_node(hvx_graph g, hvx_image in, hvx_buffer result, hvx_node* node_out);
hvx_status hvx_min_max_loc_node(hvx_graph g, hvx_image in, hvx_buffer result, hvx_buffer locations,
                                uint32_t capacity, hvx_node* node_out);
hvx_status hvx_mean_std_dev_node(hvx_graph g, hvx_image in, hvx_buffer result, hvx_node* node_out);
hvx_status hvx_equalize_hist_node(hvx_graph g, hvx_image in, hvx_image out, hvx_node* node_out);

/* User-defined local kernel (Section 5.1): `expr` over one input image a in
 * the grammar of hvx_custom_point_node, where a[dx, dy] (one-digit integer
 * offsets, |dx|, |dy| <= 2) reads the input at (x + dx, y + dy) and a alone
 * is a[0, 0].  Positions outside the image follow the node's border mode
 * (hvx_node_set_border).  The node is fused like the built-in local
 * operators; its window is read at run-time offsets by the generic kernels. */
hvx_status hvx_custom_local_node(hvx_graph g, const char* expr, hvx_image in, int out_format, hvx_image out,
                                 hvx_node* node_out);

/* Border mode of a node's inputs (default REPLICATE).  For CONSTANT the
 * value is read as the input's element type (0..255 for U8). */
hvx_status hvx_node_set_border(hvx_node node, int border, uint32_t constant_value);

/* Set one HVX_OPT_* option (the optimisations of Section 5.2 can be turned
 * off one by one); the graph is un-verified.  INVALID_PARAMETERS for an
 * unknown option or a negative tile. */
hvx_status hvx_graph_set_option(hvx_graph g, int option, int64_t value);

/* Verify and plan: checks (parameters, formats, sizes, single writer per
 * image, no cycles, bipartite node/data structure; Sections 3.1 and 5.2),
 * virtual image inference, lowering, dead-computation elimination, fusion
 * grouping and the launch plan.  No device work. */
hvx_status hvx_graph_verify(hvx_graph g);
/* Verify if needed, run on the device, and wait for completion. */
hvx_status hvx_graph_process(hvx_graph g);
/* Verify if needed and enqueue on `hip_stream` (a hipStream_t; NULL = the
 * null stream) without waiting. */
hvx_status hvx_graph_schedule(hvx_graph g, void* hip_stream);
/* Wait for the work last scheduled for this graph. */
hvx_status hvx_graph_wait(hvx_graph g);
/* Read one HVX_QUERY_* value of the verified plan.  NOT_VERIFIED before
 * verification, INVALID_PARAMETERS for an unknown attribute. */
hvx_status hvx_graph_query(hvx_graph g, int attr, int64_t* out);

/* Time candidate plans of the graph on the device and keep the fastest in
 * the context's tune cache (`iters` timed runs each; every candidate's
 * outputs must equal those of the plan in force before tuning, bit for bit,
 * else the call fails).  Candidates (Section 6.3): the fused plan, each plan
 * that cuts fusion at one value inside a fused group, the plan that cuts at
 * all of them, then the tile of each generated kernel; for a plan of one
 * hand-fused kernel, its rows per work item and XCD mapping.  The plan choice
 * is recorded under the graph's operator signature, so any graph built the
 * same way (same operators, borders, formats and sizes, same options) is
 * verified with it; the launch shape under the graph's kernel signature.
 * The graph is re-planned: batches built on it must be created again. */
hvx_status hvx_graph_autotune(hvx_graph g, void* hip_stream, int iters);
/* Tune cache as JSON text keyed by device, graph signature and size. */
hvx_status hvx_context_save_tune_cache(hvx_context ctx, const char* path);
hvx_status hvx_context_load_tune_cache(hvx_context ctx, const char* path);

/* ---- batches: many verified graphs in one kernel launch ----------------- */

/* Build a batch over n verified graphs (any mix of kinds and sizes).  The
 * work items of every graph whose plan is one hand-fused kernel go into one
 * flat work list run by a single launch (see HVX_BATCH_PERSISTENT); other
 * graphs are launched after it with their own plans.  The launches are
 * captured once into a HIP graph and replayed.  Graphs keep their image
 * pointers as of this call or of the last hvx_batch_refresh.  Graphs not yet
 * verified are verified here (their verification status on failure);
 * NOT_SUPPORTED above 65535 single-launch graphs. */
hvx_status hvx_batch_create(hvx_context ctx, const hvx_graph* graphs, uint32_t n, hvx_batch* out);
/* Re-read the graphs' image pointers (after hvx_image_swap_ptr). */
hvx_status hvx_batch_refresh(hvx_batch b);
/* Enqueue one execution of every graph in the batch on `hip_stream`. */
hvx_status hvx_batch_schedule(hvx_batch b, void* hip_stream);
/* One-shot form: create, schedule, and release once the stream is done. */
hvx_status hvx_process_batch(hvx_context ctx, const hvx_graph* graphs, uint32_t n, void* hip_stream);
/* HVX_QUERY_ALG_BYTES (bytes one schedule must move), _NUM_KERNELS (launches
 * per schedule), _NUM_OPS (work items of the single launch), _ROWS_PER_ITEM
 * (rows per work item chosen for the batch, 0 = each graph's own). */
hvx_status hvx_batch_query(hvx_batch b, int attr, int64_t* out);
/* Batch options.  HVX_BATCH_PERSISTENT (default 1): a grid sized to the
 * machine pulls chunks of work items from per-XCD atomic counters; 0: one
 * wave per work item.  HVX_BATCH_USE_GRAPH (default 1): when a schedule
 * takes more than one launch, capture them once into a HIP graph and replay
 * it (a single launch, or the legacy null stream, is launched plainly).  HVX_BATCH_ROWS (default 0): rows per
 * work item for every image of the single launch (1..65535), 0 = each
 * graph's own; it is what hvx_batch_autotune sets, and setting it pins a
 * launch shape (e.g. a tuned one) without re-tuning.  Changing an option
 * drops the capture; INVALID_PARAMETERS for an unknown option or a value out
 * of range. */
#define HVX_BATCH_PERSISTENT 1
#define HVX_BATCH_USE_GRAPH 2
#define HVX_BATCH_ROWS 3
hvx_status hvx_batch_set_option(hvx_batch b, int option, int64_t value);
/* Time candidate rows-per-work-item settings (shared by all images) and both
 * launch modes on the device (`iters` timed runs each; outputs of the first
 * and last graph checked equal across candidates); keep the fastest. */
hvx_status hvx_batch_autotune(hvx_batch b, void* hip_stream, int iters);

/* ---- serving ------------------------------------------------------------ */

#define HVX_SERVER_CONTINUOUS 0 /* admit by budget, batch admitted requests into overlapping steps */
#define HVX_SERVER_PLAIN 1      /* one request at a time: copy in, process, copy out, wait */

/* A request loop over device memory of at most hbm_budget_bytes, holding at
 * most max_slots requests on the device, using n_streams streams (>= 1). */
hvx_status hvx_server_create(hvx_context ctx, int mode, size_t hbm_budget_bytes, uint32_t max_slots,
                             uint32_t n_streams, hvx_server* out);
/* Queue a request: run verified `templ` (one non-virtual input image, one
 * non-virtual output image) on host frame `in` (row pitch in_pitch) and
 * write its output to host memory `out` (row pitch out_pitch).  Host buffers
 * must stay valid until the request is reported done.  `tag` is returned by
 * hvx_server_poll.  Templates with more images, or frames in device memory:
 * hvx_server_submit_bound. */
hvx_status hvx_server_submit(hvx_server s, hvx_graph templ, const void* in, size_t in_pitch, void* out,
                             size_t out_pitch, uint64_t tag);
/* One image of a request: the template image it stands for and the
 * request's pixels for it (host or device memory, row pitch in bytes). */
typedef struct hvx_binding {
  hvx_image image;
  void* ptr;
  size_t pitch;
} hvx_binding;
#define HVX_MEMORY_HOST 0   /* copied into device buffers from the HBM budget, outputs copied back */
#define HVX_MEMORY_DEVICE 1 /* already in device memory: the request runs on it in place */
/* Queue a request of any verified template: every non-virtual image the
 * template reads or writes is bound once in `bindings` (n entries), all in
 * the `memory` given.  Device memory needs a 16-byte aligned base and a pitch
 * that is a multiple of 64; it is read and written in place, so frames that
 * stay resident in HBM cost no copies.  Host memory is copied in (inputs)
 * and out (outputs) as in hvx_server_submit.  A template whose plan is one
 * strip kernel (edge with or without Phase, corner, Gaussian5x5, UYVY luma
 * Gaussian5x5) joins the batch launch of a step; any other template runs its
 * own plan, its intermediate images in a block taken from the HBM budget.
 * Buffers stay valid until the request is reported done.  INVALID_PARAMETERS
 * for an unbound, twice-bound or misaligned image; NOT_SUPPORTED for a
 * template with global operator results; NO_MEMORY when the request alone
 * exceeds the budget. */
hvx_status hvx_server_submit_bound(hvx_server s, hvx_graph templ, const hvx_binding* bindings, uint32_t n,
                                   int memory, uint64_t tag);
/* Collect up to `max` finished requests: tags, statuses, latencies (s, from
 * submit to completion).  Non-blocking; *n = number returned. */
hvx_status hvx_server_poll(hvx_server s, uint64_t* tags, int32_t* statuses, double* latency_s, uint32_t max,
                           uint32_t* n);
/* Block until every submitted request has finished. */
hvx_status hvx_server_drain(hvx_server s);
/* Counters: 0 submitted, 1 completed, 2 peak device bytes, 3 peak requests
 * in flight, 4 device steps launched, 5 current device bytes in use. */
hvx_status hvx_server_stats(hvx_server s, int what, int64_t* out);
/* Test hook: make the request with this tag fail (HVX_ERROR_DEVICE) without
 * running it; other requests are unaffected. */
hvx_status hvx_server_inject_failure(hvx_server s, uint64_t tag);

/* ---- release ------------------------------------------------------------ */

/* Each release invalidates the handle and sets *ref = NULL (explicit
 * release, Section 3.1).  A graph waits for its scheduled work first, a
 * batch for its last launch, a server drains its requests (a graph waits only
 * for its own schedules, not for the requests a server ran on it: release the
 * server, or drain it, before the templates it serves).  An image or
 * convolution still wired into a node of a live graph stays alive until that
 * graph (or the context) is released; a node's handle can be dropped at any
 * time, the node itself lives as long as its graph.  INVALID_PARAMETERS for a
 * NULL ref, INVALID_REFERENCE for a handle already released. */
hvx_status hvx_release_graph(hvx_graph* g);
hvx_status hvx_release_image(hvx_image* img);
hvx_status hvx_release_node(hvx_node* node);
hvx_status hvx_release_convolution(hvx_convolution* conv);
hvx_status hvx_release_batch(hvx_batch* b);
hvx_status hvx_release_server(hvx_server* s);
hvx_status hvx_release_buffer(hvx_buffer* b);

#ifdef __cplusplus
}
#endif
#endif /* HVX_H */
