// Allocation-free product entry point: gofd_apply_Ah with its grid
// workspaces in one static device array instead of buffers it would allocate.
//
// Layout of the array for one call (each part starts on a 256-byte boundary;
// b = 8 bytes per real in double precision, 4 with GOFD_FP32_GRID):
//   Y  the grid result A_FD I u      b * W^d * nrhs
//   G  the gathered field I u        b * W^d * nrhs
//   Z  spectra of the FFT passes     2b * W * (L/2) * nrhs in 2D,
//                                    2b * 4 ceil((L/2+1)/4) * W * (W + L) * nrhs in 3D
// Every part is written by the call's kernels before it is read, so nothing
// is cleared; the array keeps the last call's contents.
#include <mutex>

#include "internal.h"

namespace {

constexpr size_t WS_BYTES = (size_t)GOFD_NOALLOC_WS_BYTES;
constexpr int MAX_DEVICES = 64;

// one copy per GPU, at a different address on each
__device__ __align__(256) unsigned char scratch[WS_BYTES];

std::mutex ws_mutex;
bool ws_looked_up[MAX_DEVICES] = {};
void* ws_ptr[MAX_DEVICES] = {};

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Restores the context's workspace override when the call returns.
struct WsOverride {
  gofd_ctx_s* ctx;
  WsOverride(gofd_ctx_s* c, void* G, void* Z) : ctx(c) {
    ctx->ws_G = G;
    ctx->ws_Z = Z;
  }
  ~WsOverride() {
    ctx->ws_G = nullptr;
    ctx->ws_Z = nullptr;
  }
};

}  // namespace

void* noalloc_ws_lookup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(ws_mutex);
  if (!ws_looked_up[device]) {
    // the host-side name `scratch` is only a stand-in; the device address of
    // this GPU's copy comes from the runtime (the device is current here)
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    ws_ptr[device] = p;
    ws_looked_up[device] = true;
  }
  return ws_ptr[device];
}

extern "C" int gofd_apply_Ah_noalloc(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int nrhs, const double* u_dev,
                                     double* y_dev, int flags) {
  if (!ctx || !tr || !op || !u_dev || !y_dev || nrhs < 1) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!same_grid(tr, op)) return gofd_fail(ctx, GOFD_E_ARG, "transfer and operator use different grids");
  // the twiddle tables of the operator's period exist once the operator has
  // been built in this context; creating them here would allocate
  if (!twiddles_ready(ctx, op->L))
    return gofd_fail(ctx, GOFD_E_ARG, "operator was not created in this context");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(ws_mutex);
    if (ctx->device >= 0 && ctx->device < MAX_DEVICES && ws_looked_up[ctx->device]) base = ws_ptr[ctx->device];
  }
  if (!base) return gofd_fail(ctx, GOFD_E_HIP, "static workspace address not available on this device");
  const size_t b = (flags & GOFD_FP32_GRID) ? 4 : 8;
  const size_t nn = (size_t)tr->n_nodes;
  const size_t zc = op->d == 2 ? (size_t)op->W * (op->L / 2) : (size_t)conv3_workspace(op);
  const size_t yb = align256(b * nn * nrhs), gb = align256(b * nn * nrhs), zb = align256(2 * b * zc * nrhs);
  if (yb + gb + zb > WS_BYTES)
    return gofd_fail(ctx, GOFD_E_ARG, "gofd_apply_Ah_noalloc: " + std::to_string(nrhs) + " field(s) of this grid need " +
                                          std::to_string(yb + gb + zb) + " bytes of workspace, the static array holds " +
                                          std::to_string(WS_BYTES));
  unsigned char* p = static_cast<unsigned char*>(base);
  WsOverride ov(ctx, p + yb, p + yb + gb);
  return apply_Ah_impl(ctx, tr, op, nrhs, u_dev, y_dev, flags, p);
}
