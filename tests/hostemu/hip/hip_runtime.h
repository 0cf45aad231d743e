// Host emulation of the HIP API subset used by libladmm's sources.
//
// Test infrastructure: it lets the library's own kernels and C ABI run on the
// CPU under AddressSanitizer, so out-of-bounds indexing and launch-shape errors
// are found without a GPU.  Every GPU thread of a workgroup runs as a fiber
// (ucontext); __syncthreads() and the cross-lane operations (wavefront
// shuffles, MFMA) are barriers of the scheduler, so workgroup semantics and
// LDS contents are exact.  Workgroups run one after another.  It is never part
// of the product: the product library is built only by hipcc for gfx950.
#pragma once
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

using std::max;
using std::min;

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct float4 { float x, y, z, w; };
struct double2 { double x, y; };
struct uint4 { unsigned x, y, z, w; };
struct uint2 { unsigned x, y; };

namespace hostemu {
extern dim3 threadIdx_, blockIdx_, blockDim_, gridDim_;
void barrier();                       // workgroup barrier (also used for cross-lane ops)
int lane_id();                        // linear thread id within the workgroup
void *wave_slot(size_t bytes);        // per-thread exchange slot (lives for one exchange)
void *peer_slot(int linear_tid);      // slot of another thread of the workgroup
void launch(dim3 grid, dim3 block, std::function<void()> body);
}  // namespace hostemu

#define threadIdx (hostemu::threadIdx_)
#define blockIdx (hostemu::blockIdx_)
#define blockDim (hostemu::blockDim_)
#define gridDim (hostemu::gridDim_)

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)

inline void __syncthreads() { hostemu::barrier(); }

// ---- cross-lane operations ------------------------------------------------
template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  (void)width;
  *(T *)hostemu::wave_slot(sizeof(T)) = v;
  hostemu::barrier();
  const int me = hostemu::lane_id();
  const int other = (me & ~63) | ((me & 63) ^ mask);
  T r = *(T *)hostemu::peer_slot(other);
  hostemu::barrier();
  return r;
}

typedef float hostemu_f4 __attribute__((ext_vector_type(4)));
typedef double hostemu_d4 __attribute__((ext_vector_type(4)));

namespace hostemu {
// D = A B + C for one 16x16x4 MFMA of the wavefront containing this lane.
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; f32 output rows are
// 4 (l / 16) + r, f64 output rows l / 16 + 4 r (both checked on gfx950).
template <typename S, typename V, bool F64>
inline V mfma16(S a, S b, V c) {
  struct Slot { S a, b; };
  Slot *mine = (Slot *)wave_slot(sizeof(Slot));
  mine->a = a;
  mine->b = b;
  barrier();
  const int me = lane_id(), base = me & ~63, l = me & 63;
  V d = c;
  for (int r = 0; r < 4; ++r) {
    const int row = F64 ? (l >> 4) + 4 * r : 4 * (l >> 4) + r;
    const int col = l & 15;
    S acc = d[r];
    for (int k = 0; k < 4; ++k) {
      const Slot *pa = (const Slot *)peer_slot(base + row + 16 * k);
      const Slot *pb = (const Slot *)peer_slot(base + col + 16 * k);
      acc += pa->a * pb->b;
    }
    d[r] = acc;
  }
  barrier();
  return d;
}
}  // namespace hostemu

inline hostemu_f4 __builtin_amdgcn_mfma_f32_16x16x4f32(float a, float b, hostemu_f4 c, int, int, int) {
  return hostemu::mfma16<float, hostemu_f4, false>(a, b, c);
}
inline hostemu_d4 __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, hostemu_d4 c, int, int, int) {
  return hostemu::mfma16<double, hostemu_d4, true>(a, b, c);
}

typedef __bf16 hostemu_bf8 __attribute__((ext_vector_type(8)));

namespace hostemu {
// D = A B + C for one 16x16x32 BF16 MFMA: lane l supplies A[l % 16][8 (l / 16) + e]
// and B[8 (l / 16) + e][l % 16] (e = 0..7) and receives D[4 (l / 16) + r][l % 16].
inline hostemu_f4 mfma16_bf16(hostemu_bf8 a, hostemu_bf8 b, hostemu_f4 c) {
  struct Slot { float a[8], b[8]; };
  Slot *mine = (Slot *)wave_slot(sizeof(Slot));
  for (int e = 0; e < 8; ++e) {
    mine->a[e] = (float)a[e];
    mine->b[e] = (float)b[e];
  }
  barrier();
  const int me = lane_id(), base = me & ~63, l = me & 63;
  hostemu_f4 d = c;
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * (l >> 4) + r, col = l & 15;
    float acc = d[r];
    for (int k = 0; k < 32; ++k) {
      const Slot *pa = (const Slot *)peer_slot(base + row + 16 * (k / 8));
      const Slot *pb = (const Slot *)peer_slot(base + col + 16 * (k / 8));
      acc += pa->a[k % 8] * pb->b[k % 8];
    }
    d[r] = acc;
  }
  barrier();
  return d;
}
}  // namespace hostemu

inline hostemu_f4 __builtin_amdgcn_mfma_f32_16x16x32_bf16(hostemu_bf8 a, hostemu_bf8 b, hostemu_f4 c,
                                                          int, int, int) {
  return hostemu::mfma16_bf16(a, b, c);
}

inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
inline unsigned atomicAdd(unsigned *p, unsigned v) {
  unsigned o = *p;
  *p += v;
  return o;
}
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v) {
  unsigned long long o = *p;
  *p += v;
  return o;
}
inline unsigned long long atomicMin(unsigned long long *p, unsigned long long v) {
  unsigned long long o = *p;
  if (v < o) *p = v;
  return o;
}

// ---- runtime API ------------------------------------------------------------
typedef int hipError_t;
typedef void *hipStream_t;
typedef struct hostemu_event *hipEvent_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNoDevice = 3,
       hipErrorInvalidDevice = 4 };
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
#define hipHostMallocDefault 0

hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t);
hipError_t hipGetDeviceCount(int *);
hipError_t hipSetDevice(int);
hipError_t hipMalloc(void **, size_t);
template <typename T> hipError_t hipMalloc(T **p, size_t n) { return hipMalloc((void **)p, n); }
hipError_t hipFree(void *);
hipError_t hipHostMalloc(void **, size_t, unsigned);
template <typename T> hipError_t hipHostMalloc(T **p, size_t n, unsigned f) { return hipHostMalloc((void **)p, n, f); }
hipError_t hipHostFree(void *);
hipError_t hipMemcpy(void *, const void *, size_t, hipMemcpyKind);
hipError_t hipMemcpyAsync(void *, const void *, size_t, hipMemcpyKind, hipStream_t);
hipError_t hipMemsetAsync(void *, int, size_t, hipStream_t);
hipError_t hipStreamCreate(hipStream_t *);
#define hipStreamNonBlocking 0x01
hipError_t hipStreamCreateWithFlags(hipStream_t *, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipEventCreate(hipEvent_t *);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float *, hipEvent_t, hipEvent_t);
// A file-scope __device__ array is a host array here; its address is its symbol's.
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
  *p = const_cast<void *>(symbol);
  return hipSuccess;
}

// Stream capture: kernel launches of the capturing thread are recorded into the
// graph and run, in order, at each hipGraphLaunch.  Any other stream operation
// while capturing is an error here, so a copy, fill or event that slipped into
// a captured region fails the emulated run.
typedef struct hostemu_graph *hipGraph_t;
typedef struct hostemu_graph *hipGraphExec_t;
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal,
                            hipStreamCaptureModeRelaxed };
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode);
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *);
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, void *, char *, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphDestroy(hipGraph_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);

#define hipLaunchKernelGGL(K, G, B, SH, S, ...)                    \
  do {                                                            \
    (void)(SH);                                                   \
    (void)(S);                                                    \
    hostemu::launch(dim3(G), dim3(B), [=]() { K(__VA_ARGS__); }); \
  } while (0)
