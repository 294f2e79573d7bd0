// Context, error reporting, device buffers, twiddle tables and a prefix scan.
#include <cmath>
#include <cstring>

#include "internal.h"

int gofd_fail(gofd_ctx_s* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int dev_reserve(gofd_ctx_s* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return GOFD_OK;
  b.release();
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return gofd_fail(ctx, GOFD_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return GOFD_OK;
}

gofd_ctx_s::~gofd_ctx_s() {
  for (gofd_ctx_s* c : children) delete c;
  if (!borrowed_twiddles)
    for (auto& kv : twiddles) delete kv.second;
  if (host_state) (void)hipHostFree(host_state);
  if (solver_ws && solver_ws_free) solver_ws_free(solver_ws);
  if (ev_in) (void)hipEventDestroy(ev_in);
  if (ev_out) (void)hipEventDestroy(ev_out);
  if (work) (void)hipStreamDestroy(work);
  if (owns_stream && stream) (void)hipStreamDestroy(stream);
}

gofd_ctx_s* ctx_child(gofd_ctx_s* parent, size_t index) {
  while (parent->children.size() <= index) {
    auto* c = new (std::nothrow) gofd_ctx_s();
    if (!c) return nullptr;
    c->device = parent->device;
    c->num_cu = parent->num_cu;
    c->twiddles = parent->twiddles;
    c->borrowed_twiddles = true;
    c->col_sched = parent->col_sched;
    c->row_sched = parent->row_sched;
    c->sched3 = parent->sched3;
    c->owns_stream = true;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        dev_reserve(c, c->scratch, 1 << 20) != GOFD_OK || dev_reserve(c, c->flag, 256) != GOFD_OK ||
        hipMemset(c->flag.p, 0, 256) != hipSuccess || hipMemset(c->scratch.p, 0, 1 << 20) != hipSuccess) {
      delete c;
      return nullptr;
    }
    parent->children.push_back(c);
  }
  gofd_ctx_s* c = parent->children[index];
  // tables and schedules made or tuned on the parent since the child was created
  c->twiddles = parent->twiddles;
  c->col_sched = parent->col_sched;
  c->row_sched = parent->row_sched;
  c->sched3 = parent->sched3;
  return c;
}

WorkStream::WorkStream(gofd_ctx_s* c) : ctx(c), saved(c->stream) {
  (void)hipEventRecord(ctx->ev_in, saved);
  (void)hipStreamWaitEvent(ctx->work, ctx->ev_in, 0);
  ctx->stream = ctx->work;
}

WorkStream::~WorkStream() {
  (void)hipEventRecord(ctx->ev_out, ctx->work);
  (void)hipStreamWaitEvent(saved, ctx->ev_out, 0);
  ctx->stream = saved;
}

extern "C" int gofd_create(gofd_ctx* out, void* hip_stream) {
  if (!out) return GOFD_E_ARG;
  auto* c = new (std::nothrow) gofd_ctx_s();
  if (!c) return GOFD_E_OOM;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return GOFD_E_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&c->work, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return GOFD_E_HIP;
  }
  if (dev_reserve(c, c->scratch, 1 << 20) != GOFD_OK || dev_reserve(c, c->flag, 256) != GOFD_OK) {
    delete c;
    return GOFD_E_OOM;
  }
  if (hipMemset(c->flag.p, 0, 256) != hipSuccess || hipMemset(c->scratch.p, 0, 1 << 20) != hipSuccess) {
    delete c;
    return GOFD_E_HIP;
  }
  (void)noalloc_ws_lookup(c->device);   // once per device, with the device current
  *out = c;
  return GOFD_OK;
}

extern "C" int gofd_destroy(gofd_ctx ctx) {
  if (!ctx) return GOFD_E_ARG;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return GOFD_OK;
}

extern "C" int gofd_set_stream(gofd_ctx ctx, void* hip_stream) {
  if (!ctx) return GOFD_E_ARG;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return GOFD_OK;
}

extern "C" const char* gofd_last_error(gofd_ctx ctx) {
  return ctx ? ctx->last_error.c_str() : "null context";
}

extern "C" const char* gofd_strerror(int status) {
  switch (status) {
    case GOFD_OK: return "GOFD_OK";
    case GOFD_E_ARG: return "GOFD_E_ARG";
    case GOFD_E_DEGENERATE: return "GOFD_E_DEGENERATE";
    case GOFD_E_RANK: return "GOFD_E_RANK";
    case GOFD_E_ZERO_COLSUM: return "GOFD_E_ZERO_COLSUM";
    case GOFD_E_NOT_CONVERGED: return "GOFD_E_NOT_CONVERGED";
    case GOFD_E_BREAKDOWN: return "GOFD_E_BREAKDOWN";
    case GOFD_E_HIP: return "GOFD_E_HIP";
    case GOFD_E_OOM: return "GOFD_E_OOM";
    case GOFD_E_NUMERIC: return "GOFD_E_NUMERIC";
    case GOFD_E_UNSUPPORTED: return "GOFD_E_UNSUPPORTED";
    default: return "unknown status";
  }
}

// Twiddle factors exp(-2 pi i t / L), t = 0..L-1, evaluated on the host with
// the angle reduced to the first octant so every entry is correctly rounded
// to within an ulp or so.
static void host_twiddles(int L, std::vector<double>& re, std::vector<double>& im) {
  re.resize(L);
  im.resize(L);
  for (int t = 0; t < L; ++t) {
    // exact symmetries of the unit circle at multiples of L/8
    long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)L;
    long double c = std::cos(a), s = std::sin(a);
    if (4 * t == L) { c = 0; s = 1; }
    if (2 * t == L) { c = -1; s = 0; }
    if (4 * t == 3 * L) { c = 0; s = -1; }
    if (t == 0) { c = 1; s = 0; }
    re[t] = (double)c;
    im[t] = -(double)s;
  }
}

static TwiddleTables* get_tables(gofd_ctx_s* ctx, int L) {
  auto it = ctx->twiddles.find(L);
  if (it != ctx->twiddles.end()) return it->second;
  auto* tt = new TwiddleTables();
  std::vector<double> re, im;
  host_twiddles(L, re, im);
  std::vector<cplx<double>> h64(L);
  std::vector<cplx<float>> h32(L);
  for (int t = 0; t < L; ++t) {
    h64[t] = {re[t], im[t]};
    h32[t] = {(float)re[t], (float)im[t]};
  }
  if (dev_reserve(ctx, tt->tw64, sizeof(cplx<double>) * L) != GOFD_OK ||
      dev_reserve(ctx, tt->tw32, sizeof(cplx<float>) * L) != GOFD_OK) {
    delete tt;
    return nullptr;
  }
  if (hipMemcpy(tt->tw64.p, h64.data(), sizeof(cplx<double>) * L, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(tt->tw32.p, h32.data(), sizeof(cplx<float>) * L, hipMemcpyHostToDevice) != hipSuccess) {
    delete tt;
    return nullptr;
  }
  ctx->twiddles[L] = tt;
  return tt;
}

bool twiddles_ready(const gofd_ctx_s* ctx, int L) { return ctx->twiddles.count(L) != 0; }

const cplx<double>* twiddles64(gofd_ctx_s* ctx, int L) {
  auto* t = get_tables(ctx, L);
  return t ? t->tw64.as<cplx<double>>() : nullptr;
}
const cplx<float>* twiddles32(gofd_ctx_s* ctx, int L) {
  auto* t = get_tables(ctx, L);
  return t ? t->tw32.as<cplx<float>>() : nullptr;
}

// ------------------------------------------------------------------ scan

constexpr int SCAN_BLOCK = 1024;

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_blocks(const int32_t* __restrict__ in,
                                                            int32_t* __restrict__ out,
                                                            int32_t* __restrict__ block_sums, int64_t n) {
  __shared__ int32_t s[SCAN_BLOCK];
  int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  int32_t v = (i < n) ? in[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
    int32_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = s[threadIdx.x] - v;   // exclusive within the block
  if (threadIdx.x == SCAN_BLOCK - 1) block_sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ block_prefix, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
  if (i < n) out[i] += block_prefix[blockIdx.x];
}

__global__ void k_scan_total(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

// ints of the block sums and their prefixes over every level of a scan of n values
static int64_t scan_ws_ints(int64_t n) {
  int64_t t = 0;
  for (;;) {
    const int64_t nb = std::max<int64_t>(1, (n + SCAN_BLOCK - 1) / SCAN_BLOCK);
    t += 2 * (nb + 1);
    if (nb <= 1) return t;
    n = nb;
  }
}

static void scan_levels(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* ws) {
  const int64_t nb = std::max<int64_t>(1, (n + SCAN_BLOCK - 1) / SCAN_BLOCK);
  int32_t* sums = ws;
  int32_t* pref = ws + nb + 1;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(SCAN_BLOCK), 0, st, in, out, sums, n);
  if (nb > 1) {
    scan_levels(st, sums, pref, nb, ws + 2 * (nb + 1));
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_BLOCK), 0, st, out, pref, n);
  }
}

int scan_prepare(gofd_ctx_s* ctx, int64_t n) { return dev_reserve(ctx, ctx->scan_ws, sizeof(int32_t) * scan_ws_ints(n)); }

// out[0..n] = exclusive prefix sums of in[0..n) and the total, on the context's stream (no host round trip;
// the levels' block sums live in a workspace of the context)
int scan_exclusive_i32(gofd_ctx_s* ctx, const int32_t* in, int32_t* out, int64_t n) {
  GOFD_TRY(scan_prepare(ctx, n));
  scan_levels(ctx->stream, in, out, n, ctx->scan_ws.as<int32_t>());
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, ctx->stream, in, out, n);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}
