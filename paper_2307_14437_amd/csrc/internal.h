// Internal declarations of the GoFD HIP library (gfx950).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "cg_items.h"
#include "cg_state.h"

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "gofd.h"

// ------------------------------------------------------------------ errors

#define GOFD_TRY(expr)                  \
  do {                                  \
    int _st = (expr);                   \
    if (_st != GOFD_OK) return _st;     \
  } while (0)

#define HIP_TRY(ctx, expr)                                                         \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return gofd_fail((ctx), GOFD_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

struct gofd_ctx_s;
int gofd_fail(gofd_ctx_s* ctx, int code, const std::string& msg);

// ------------------------------------------------------------------ complex

template <typename R>
struct cplx {
  R x, y;
};

// ------------------------------------------------------------------ device buffer

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// grow-only allocation; returns GOFD_OK / GOFD_E_OOM
int dev_reserve(gofd_ctx_s* ctx, DevBuf& b, size_t bytes);

// ------------------------------------------------------------------ context

struct TwiddleTables {
  DevBuf tw64;   // cplx<double>[L], exp(-2 pi i t / L)
  DevBuf tw32;   // cplx<float>[L]
};

struct gofd_ctx_s {
  hipStream_t stream = nullptr;      // the caller's stream (may be the null stream)
  hipStream_t work = nullptr;        // library stream for solves (capturable into graphs)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int device = 0;
  int num_cu = 256;
  std::string last_error;
  std::map<int, TwiddleTables*> twiddles;   // keyed by L
  std::map<std::pair<int, bool>, int> col_sched;   // column-pass schedule per (L, FP32), see gofd_autotune
  std::map<std::pair<int, bool>, int> row_sched;   // 2D first row pass of the products: values per thread
  std::map<std::pair<int, bool>, int> sched3;      // 3D y/z/y passes: 0 default, 1 two slots per block
  DevBuf scratch;                           // small reduction scratch (partials, counters)
  DevBuf scan_ws;                           // block sums of the prefix-sum helper
  DevBuf flag;                              // int status flags
  // When set, the next kernel launched through GOFD_LAUNCH records these
  // events at its own start and end (stage timing); the launch clears them.
  hipEvent_t timer_start = nullptr, timer_stop = nullptr;
  // page-locked host copies of the CG state (two chunk slots, written by the
  // last iteration of each chunk, and one for a residual replacement): the
  // host reads one check's state while the next chunk of iterations runs
  void* host_state = nullptr;
  // the solver's device workspace (CG vectors, grid, partial slots, ...),
  // kept from one solve to the next so that a solve allocates only when it
  // needs more than the last one
  void* solver_ws = nullptr;
  void (*solver_ws_free)(void*) = nullptr;
  size_t host_state_bytes = 0;
  // Workspace override: while set (by gofd_apply_Ah_noalloc, for the length
  // of one call), the products take the gathered field I u from ws_G and the
  // spectra of the FFT passes from ws_Z instead of reserving the operator's
  // buffers, so that they allocate nothing
  void* ws_G = nullptr;
  void* ws_Z = nullptr;
  // Child contexts of a batched solve whose problems have several grid
  // shapes: one per shape group, each with its own streams, solver
  // workspace and page-locked state, so the groups run concurrently from
  // host threads.  A child borrows the parent's twiddle tables and column
  // schedules; children are kept for later calls and freed with the parent.
  std::vector<gofd_ctx_s*> children;
  bool borrowed_twiddles = false;
  bool owns_stream = false;          // a child's stream (created with it)
  ~gofd_ctx_s();
};

// A child context for concurrent work on the parent's device (see children).
gofd_ctx_s* ctx_child(gofd_ctx_s* parent, size_t index);

// Launch on a stream; if the context holds a pending pair of timing events,
// the launch records them at the kernel's start and end (AMD extended launch).
#define GOFD_LAUNCH(CTX, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                               \
  do {                                                                                                          \
    if ((CTX)->timer_start) {                                                                                   \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, (CTX)->timer_start, (CTX)->timer_stop, 0,        \
                            __VA_ARGS__);                                                                       \
      (CTX)->timer_start = (CTX)->timer_stop = nullptr;                                                         \
    } else {                                                                                                    \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                                      \
    }                                                                                                           \
  } while (0)

// Run a solve on the library's own stream, ordered after the caller's stream
// on entry and before it on exit.
struct WorkStream {
  gofd_ctx_s* ctx;
  hipStream_t saved;
  explicit WorkStream(gofd_ctx_s* c);
  ~WorkStream();
};

const cplx<double>* twiddles64(gofd_ctx_s* ctx, int L);
const cplx<float>* twiddles32(gofd_ctx_s* ctx, int L);
// whether the twiddle tables of period L already exist (no allocation)
bool twiddles_ready(const gofd_ctx_s* ctx, int L);
// Device address of the allocation-free entry point's static workspace on the
// context's device, looked up once per device at context creation; nullptr
// if the lookup failed (the entry point then reports GOFD_E_HIP).
void* noalloc_ws_lookup(int device);

// ------------------------------------------------------------------ handles

struct gofd_transfer_s {
  int d = 2, N = 0, W = 0;
  double R = 1.0, center[3] = {0, 0, 0};
  double h = 0.0, lo[3] = {0, 0, 0};
  int64_t nv = 0, ne = 0, n_nodes = 0, nnz = 0;
  DevBuf X;          // double[nv*d]
  DevBuf elems;      // int32[ne*(d+1)]
  DevBuf elem;       // int32[n_nodes], element of each node or -1
  DevBuf rec;        // ElemRec2/ElemRec3[ne]: affine barycentric map per element
  DevBuf csc_off;    // int32[nv+1]
  DevBuf csc_node;   // int32[nnz]
  DevBuf csc_w;      // double[nnz]
  DevBuf csc_w32;    // float[nnz]
  DevBuf D;          // double[nv]
  DevBuf dscale;     // double[nv]: 1/D_j (0 where D_j == 0)
  DevBuf dsqrt;      // double[nv]: 1/sqrt(D_j) (0 where D_j == 0)
  DevBuf bmask;      // uint8[nv], 1 = Dirichlet vertex
  DevBuf imask;      // double[nv], 1.0 interior, 0.0 Dirichlet
  DevBuf ell_idx;    // 3D: int32[n_nodes+1], compact row of each inside node or -1
  DevBuf ell_v;      // 3D: int32[n_inside*4], vertex ids of the interpolation row
  DevBuf ell_w;      // 3D: double[n_inside*4], barycentric weights (same bits as the CSC)
  DevBuf row32_v;    // 2D: int4[n_nodes]: vertex ids of each node's row and the bits of weight 0
  DevBuf row32_w;    // 2D: float2[n_nodes]: weights 1 and 2 (all rounded like csc_w32; zero outside)
  // 2D row-pair form of I^T (the last row pass sums each vertex's entries in
  // its rows; see build_rowpairs): present when rp_ok
  bool rp_ok = false;
  bool seg_rows_ok = false;   // seg_row / rp_pos present (at most three entries per node)
  int64_t n_slots = 0;  // partial sums: one per (vertex, row pair) with entries
  int rp_ent_ahead = 0;   // entries per thread the last row pass reads ahead (16, 24 or 32: not above the median count)
  DevBuf rp_meta;    // int4[pairs]: entry base, entries per thread, segment base, segments
  DevBuf rp_tseg;    // int32[pairs * threads]: first segment of each thread | its entry count << 16
  DevBuf rp_code;    // uint16[...]: local node (2 rows) | end-of-segment flag, thread-interleaved
  DevBuf rp_w32;     // float[...]: weights (csc_w32 values), same layout
  DevBuf rp_w64;     // double[...]: weights (csc_w values)
  DevBuf rp_dest;    // int32[segments]: partial slot of each segment (vertex-major)
  DevBuf pv_off;     // int32[nv + 1]: partial slots of each vertex
  // the FP32 gather through the segments: the slot values of a row pair are
  // staged in LDS, and each node reads its (up to) three from there
  DevBuf rp_pos;     // int32[segments]: row-pair-major position of each slot (inverse of rp_dest)
  DevBuf seg_row;    // int4[n_nodes]: local segment of corners 0 | 1 << 16, corner 2, bits of weights 0 and 1
  DevBuf seg_row_w2; // float[n_nodes]: weight of corner 2 (weights as in rp_w32; zero outside)
  std::vector<int32_t> elems_host;
  std::vector<uint8_t> bmask_host;
  std::vector<double> X_host;
  gofd_transfer_info info{};
  gofd_ctx_s* ctx = nullptr;
};

struct gofd_fdop_s {
  int d = 2, N = 0, W = 0, L = 0, half = 0;
  double s = 0.5, h = 0.0, h2s = 1.0, R = 1.0, center[3] = {0, 0, 0};
  std::vector<double> T_host;   // octant (W^d)
  DevBuf T;                     // double[W^d]
  DevBuf That64;                // double[half^d], includes the 1/L^d normalisation
  DevBuf That32;                // float [half^d]
  DevBuf Z;                     // spectra workspace
  DevBuf G;                     // gathered grid field (I u) workspace
  DevBuf Y;                     // grid-field workspace
  gofd_ctx_s* ctx = nullptr;
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2); renumber them so that logically adjacent blocks share an XCD, which
// keeps a kernel's reads of neighbouring data in one L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int per = n / 8, rem = n % 8;
  const int x = b % 8, i = b / 8;
  const int start = (x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
  return start + i;
}

// Global-memory view of a device pointer.  Pointers read from descriptors in
// memory are generic to the compiler, whose loads through them become flat
// instructions that the wave must track on two counters; through this view
// they are global loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Loads of 16-byte vectors through a global view (the HIP vector classes
// cannot be copied from a qualified address space; the builtin vector types can)
typedef int gint4_t __attribute__((ext_vector_type(4)));
typedef double gdouble2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int4 gload(const int4* p, long long i) {
  const gint4_t v = gmem(reinterpret_cast<const gint4_t*>(p))[i];
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 gload(const double2* p, long long i) {
  const gdouble2_t v = gmem(reinterpret_cast<const gdouble2_t*>(p))[i];
  return make_double2(v.x, v.y);
}
typedef float gfloat2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gload(const float2* p, long long i) {
  const gfloat2_t v = gmem(reinterpret_cast<const gfloat2_t*>(p))[i];
  return make_float2(v.x, v.y);
}

// ------------------------------------------------------------------ internal API

// Exclusive scan of int32 counts (n entries) into out (n+1 entries).
int scan_exclusive_i32(gofd_ctx_s* ctx, const int32_t* in, int32_t* out, int64_t n);
// reserve the scan's workspace for n values ahead of time (so that a timed scan allocates nothing)
int scan_prepare(gofd_ctx_s* ctx, int64_t n);

// Grid-space convolution y = A_FD v for fields on the grid; `src` selects how
// the field is produced (from a grid array or gathered from vertex values).
struct GatherSpec {
  // gather v = I u: all pointers device; u has nrhs*nv entries (stride nv)
  const gofd_transfer_s* tr = nullptr;
  const double* u = nullptr;
  const double* col_scale = nullptr;   // optional per-vertex scale applied to u (D^{-1/2})
  const double* mask = nullptr;        // optional per-vertex mask (interior)
  const int* skip = nullptr;           // optional per-rhs flag (stride skip_stride ints): rhs already finished
  int skip_stride = 0;
  bool pregathered = false;            // the grid field I u is already in the operator's G workspace
  double* dpart = nullptr;             // optional: per-block partials (gamma, (r, r), (A v, v)) of the column pass
  gofd_cg::Level1 lv1;                 // level-1 partials of gamma and (r, r) the column pass sums up
  gofd_cg::Finish fin;                 // optional: CG reductions finished by the last pass
  // batched mode: item blockIdx.y gathers from items[it] (its mesh) at ubase + off
  const CgItem* items = nullptr;
  const double* ubase = nullptr;
  bool items_mask = false;             // multiply by the item's interior mask
  const void* const* that64_tab = nullptr;   // per-item spectrum of the embedded kernel (device tables)
  const void* const* that32_tab = nullptr;
  // 2D batches whose transfers have the row-pair form of I^T: pass C sums
  // the segments into the partial slots (item it at rp_P + it * rp_pstride)
  // instead of writing the grid field
  double* rp_P = nullptr;
  long long rp_pstride = 0;
  int rp_ent_ahead = 0;                // entries per thread read ahead (the largest choice of the items)
  // with rp_us as well (every item has seg_row): the FP32 gather reads the
  // vector's values per slot (item it at rp_us + it * rp_pstride, row-pair-major
  // positions) instead of per vertex
  const float* rp_us = nullptr;
  // optional list of the items still iterating: the launches cover nrhs
  // items, block row y working on item amap[y] (workspaces stay per item)
  const int* amap = nullptr;
};

// Apply A_FD with the FFT embedding: input either a grid field (v != nullptr,
// nrhs*W^d doubles) or a gather spec; output grid field y (double or float,
// nrhs*W^d).  fp32 selects the single-precision pipeline.
// passes: bit mask of the kernels to launch (1: pass A, 2: pass B, 4: pass C,
// 8: the gather I u when g is given, into the operator's G workspace), 15 = all.
// FFT period of the embedding for a grid of half-width N, and the threads
// and row pairs per block of the row passes for period L
int conv_period(int N);
// whether the batched gather of conv_apply runs inside the first row pass
// (passes 8 and 1 together; 2D, FP32 pipeline, from the per-node rows)
bool conv_gather_fused(const gofd_fdop_s* op, bool fp32);
int conv_rowpass_threads(int L);
int conv_rowpass_lines(int L);
// Row-pair I^T form: capacity (doubles) of the per-block segment sums;
// entries per thread the last row pass fetches ahead (the entry arrays carry
// that many rows of padding); 16-bit entry code: local node in the low 15
// bits, RP_END on the last entry of a segment (padding: node 0, weight 0)
constexpr int RP_SEGCAP = 2048;
constexpr int RP_EPRE = 32;
constexpr int RP_NODE = 0x7fff;
constexpr int RP_END = 0x8000;

int conv_apply(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const double* v, const GatherSpec* g,
               void* y, bool fp32, int passes = 15);

bool same_grid(const gofd_transfer_s* tr, const gofd_fdop_s* op);

// A_h u and its variants (the flags of gofd_apply_Ah); ygrid: workspace for
// the grid result A_FD I u (nrhs fields of W^d values in the grid precision),
// or nullptr to use the operator's buffer.
int apply_Ah_impl(gofd_ctx_s* ctx, gofd_transfer_s* tr, gofd_fdop_s* op, int nrhs, const double* u, double* y,
                  int flags, void* ygrid);

// Number of blocks of the column pass (one partial of (A v, v) each; in 3D
// the z-line pass).
int conv_passB_blocks(const gofd_fdop_s* op, bool fp32);

// 3D product on grid fields (v64 or v32 source, nrhs fields of W^3 values);
// passes: 1 x forward, 2 y/z/y passes, 4 x inverse.  Workspace op->Z holds
// conv3_workspace(op) complex values per rhs.
int conv3_run(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const double* v64, const float* v32, void* y, bool fp32,
              int passes, const int* skip_flag, int skip_stride, double* dpart, const gofd_cg::Level1& lv1,
              const gofd_cg::Finish& fin, const void* const* that_tab = nullptr, const int* amap = nullptr);
long long conv3_workspace(const gofd_fdop_s* op);
// Time the 3D y/z/y passes in both schedules on a zero field of the grid,
// install the faster in ctx->sched3; returns it (0 or 1) or an error.
int conv3_tune(gofd_ctx_s* ctx, const gofd_grid* grid, bool fp32, double* times);
int conv3_passC_blocks(const gofd_fdop_s* op, bool fp32);

// Reserve the spectra workspace and twiddle tables for nrhs fields, so that
// later products allocate nothing (required inside graph capture).
int conv_prepare(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs);

// z_j = scale_j * sum_k w_kj y_k over the CSC structure (I^T y), optionally
// masked; y is double or float (fp32).  nrhs fields.
int scatter_apply(gofd_ctx_s* ctx, const gofd_transfer_s* tr, int nrhs, const void* y, bool fp32,
                  const double* scale, const double* mask, double* z);

int fdop_init_geometry(gofd_ctx_s* ctx, gofd_fdop_s* op, double s, const gofd_grid* grid);

// Compute the spectral multiplier of the circulant embedding from T (device).
int fdop_finish(gofd_ctx_s* ctx, gofd_fdop_s* op);
