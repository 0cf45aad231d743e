// Fiber scheduler and runtime API of the host emulation (see hip/hip_runtime.h).
#include "hip/hip_runtime.h"

#include <ucontext.h>

#include <memory>

namespace hostemu {

dim3 threadIdx_, blockIdx_, blockDim_, gridDim_;

namespace {

constexpr size_t kStack = 256 * 1024;
constexpr size_t kSlot = 64;

struct Fiber {
  ucontext_t ctx;
  std::unique_ptr<char[]> stack;
  dim3 tid;
  int linear = 0;
  bool done = false;
  bool waiting = false;
  alignas(16) unsigned char slot[kSlot];
};

ucontext_t g_sched;
std::vector<Fiber> *g_fibers = nullptr;
Fiber *g_cur = nullptr;
std::function<void()> *g_body = nullptr;

void entry() {
  (*g_body)();
  g_cur->done = true;
  swapcontext(&g_cur->ctx, &g_sched);
}

void switch_to(Fiber &f) {
  g_cur = &f;
  threadIdx_ = f.tid;
  swapcontext(&g_sched, &f.ctx);
}

}  // namespace

void barrier() {
  g_cur->waiting = true;
  swapcontext(&g_cur->ctx, &g_sched);
}

int lane_id() { return g_cur->linear; }
void *wave_slot(size_t bytes) {
  if (bytes > kSlot) abort();
  return g_cur->slot;
}
void *peer_slot(int linear_tid) { return (*g_fibers)[linear_tid].slot; }

}  // namespace hostemu

struct hostemu_graph {
  struct Node { dim3 grid, block; std::function<void()> body; };
  std::vector<Node> nodes;
};

namespace hostemu {
namespace {
thread_local hostemu_graph *g_capture = nullptr;
}

void launch(dim3 grid, dim3 block, std::function<void()> body) {
  if (g_capture) {
    g_capture->nodes.push_back({grid, block, std::move(body)});
    return;
  }
  gridDim_ = grid;
  blockDim_ = block;
  const int nthr = (int)(block.x * block.y * block.z);
  std::vector<Fiber> fibers(nthr);
  for (auto &f : fibers) f.stack.reset(new char[kStack]);
  g_fibers = &fibers;
  g_body = &body;
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        blockIdx_ = dim3(bx, by, bz);
        for (int t = 0; t < nthr; ++t) {
          Fiber &f = fibers[t];
          f.linear = t;
          f.tid = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
          f.done = f.waiting = false;
          getcontext(&f.ctx);
          f.ctx.uc_stack.ss_sp = f.stack.get();
          f.ctx.uc_stack.ss_size = kStack;
          f.ctx.uc_link = nullptr;
          makecontext(&f.ctx, entry, 0);
        }
        for (;;) {
          int live = 0;
          for (auto &f : fibers) {
            if (f.done) continue;
            f.waiting = false;
            switch_to(f);
            if (!f.done) ++live;
          }
          if (!live) break;   // every thread finished; otherwise all reached the barrier
        }
      }
  g_fibers = nullptr;
}

}  // namespace hostemu

// ---- runtime API ------------------------------------------------------------
struct hostemu_event { std::chrono::steady_clock::time_point t; };

hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "success" : "emulated error"; }
hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorNoDevice; }
hipError_t hipMalloc(void **p, size_t n) {
  // filled with a pattern so reads of memory no kernel wrote stand out
  *p = aligned_alloc(256, (n + 255) / 256 * 256);
  if (!*p) return hipErrorOutOfMemory;
  memset(*p, 0xCD, n);
  return hipSuccess;
}
hipError_t hipFree(void *p) { free(p); return hipSuccess; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void *p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
  if (hostemu::g_capture) return hipErrorInvalidValue;
  return hipMemcpy(d, s, n, k);
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
  if (hostemu::g_capture) return hipErrorInvalidValue;
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t *s) { *s = (hipStream_t)0x1; return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t)0x2; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hostemu::g_capture ? hipErrorInvalidValue : hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = new hostemu_event(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  if (hostemu::g_capture) return hipErrorInvalidValue;
  e->t = std::chrono::steady_clock::now();
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  if (hostemu::g_capture) return hipErrorInvalidValue;
  hostemu::g_capture = new hostemu_graph();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) {
  if (!hostemu::g_capture) return hipErrorInvalidValue;
  *g = hostemu::g_capture;
  hostemu::g_capture = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, void *, char *, size_t) {
  *e = new hostemu_graph(*g);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  if (hostemu::g_capture) return hipErrorInvalidValue;
  for (auto &n : e->nodes) hostemu::launch(n.grid, n.block, n.body);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
  return hipSuccess;
}
