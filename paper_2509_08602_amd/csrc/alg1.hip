// Algorithm 1 (overlapping low-dose point sampling, Sec. 2.C.2) on the device,
// integer exact, and the low-dose band of Sec. 2.C.1.
//
// Sets of voxels are bitsets: bit v % 64 of word v / 64.  Algorithm 1 is
// sequential over the plans (each plan thins the running union of the points
// before it), so one workgroup of 1024 threads runs the whole algorithm; the
// work inside each plan step (popcounts, hashing, the two radix selections,
// the set algebra) is spread over the workgroup.
//
// Conventions of the selection (the paper says only "randomly select"):
//   counts:  round-half-even of (N_LD,j / |V_j|) * |X| in IEEE double, clamped;
//   order:   plans by decreasing density min(1, N_LD,j / |V_j|), ties by index;
//   choice:  the K members of X with the smallest (h(seed, step, v), v), with
//            step 2 r for the thinning and 2 r + 1 for the new region of the
//            plan at rank r, h(s, t, v) = sm(sm(sm(s) ^ t) ^ v) and sm the
//            SplitMix64 output function.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "kernels.h"

namespace ladmm {

// Scratch of the allocation-free Algorithm 1 entry point: one file-scope
// device array per device, never freed.  In host code its name is a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per device
// with that device current, and only that address is handed to kernels and
// copies.
namespace {
constexpr size_t kAlg1ScratchBytes = (size_t)32 << 20;   // 32 MiB
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kAlg1ScratchBytes];
std::mutex g_scratch_mu[kMaxDevices];
unsigned char *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t alg1_scratch_bytes() { return kAlg1ScratchBytes; }

std::mutex *alg1_scratch_lock(int device) {
  return device >= 0 && device < kMaxDevices ? &g_scratch_mu[device] : nullptr;
}

// The device address of `scratch` on `device` (which must be current); the
// caller holds alg1_scratch_lock(device).
hipError_t alg1_scratch(int device, unsigned char **ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (unsigned char *)p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

namespace {

constexpr int kThreads = 1024;

__device__ __forceinline__ uint64_t sm64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ int64_t block_sum_i64(int64_t v, int64_t *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  int64_t r = 0;
  for (int w = 0; w < kThreads / 64; ++w) r += sh[w];
  __syncthreads();
  return r;   // every thread gets the total
}

__device__ int64_t popcount_set(const uint64_t *a, int W, int64_t *sh) {
  int64_t c = 0;
  for (int w = threadIdx.x; w < W; w += kThreads) c += __popcll(a[w]);
  return block_sum_i64(c, sh);
}

// round-half-even((n_ld / vol) * set) clamped to [0, set], IEEE double.
__device__ int64_t target_count(int32_t n_ld, int64_t vol, int64_t set) {
  const double omega = fmin(1.0, (double)n_ld / (double)vol);
  const double c = rint(omega * (double)set);
  return (int64_t)fmin((double)set, c);
}

// out = the `count` members of S with the smallest (key, voxel); S has `size`
// members.  keys: scratch of W * 64 uint64.  tmp: scratch bitset of W words.
__device__ void select_smallest(const uint64_t *S, int64_t size, int64_t count, int W,
                                uint64_t base, uint64_t *out, uint64_t *keys, uint64_t *tmp,
                                int64_t *sh, uint32_t *hist) {
  if (count <= 0) {
    for (int w = threadIdx.x; w < W; w += kThreads) out[w] = 0;
    __syncthreads();
    return;
  }
  if (count >= size) {
    for (int w = threadIdx.x; w < W; w += kThreads) out[w] = S[w];
    __syncthreads();
    return;
  }
  // keys of the members
  for (int w = threadIdx.x; w < W; w += kThreads) {
    uint64_t word = S[w];
    while (word) {
      const int b = __ffsll((unsigned long long)word) - 1;
      word &= word - 1;
      const uint64_t v = (uint64_t)w * 64 + b;
      keys[v] = sm64(v ^ base);
    }
  }
  __syncthreads();
  // radix select of the count-th smallest key, 8 bits per pass from the top
  uint64_t prefix = 0, pmask = 0;
  int64_t need = count;     // rank (1-based) still to find among keys matching prefix
  int64_t below = 0;        // members with key < prefix-range start
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += kThreads) hist[i] = 0;
    __syncthreads();
    for (int w = threadIdx.x; w < W; w += kThreads) {
      uint64_t word = S[w];
      while (word) {
        const int b = __ffsll((unsigned long long)word) - 1;
        word &= word - 1;
        const uint64_t key = keys[(uint64_t)w * 64 + b];
        if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t acc = 0;
      int d = 0;
      for (; d < 256; ++d) {
        if (acc + (int64_t)hist[d] >= need) break;
        acc += hist[d];
      }
      sh[0] = d;
      sh[1] = acc;
    }
    __syncthreads();
    const int d = (int)sh[0];
    const int64_t acc = sh[1];
    __syncthreads();
    need -= acc;
    below += acc;
    prefix |= (uint64_t)d << shift;
    pmask |= (uint64_t)255 << shift;
  }
  // prefix is the threshold key T; `below` members have key < T and `need`
  // members with key == T are taken, in increasing voxel order.
  for (int w = threadIdx.x; w < W; w += kThreads) {
    uint64_t word = S[w], lo = 0, eq = 0;
    while (word) {
      const int b = __ffsll((unsigned long long)word) - 1;
      word &= word - 1;
      const uint64_t key = keys[(uint64_t)w * 64 + b];
      if (key < prefix) lo |= 1ull << b;
      else if (key == prefix) eq |= 1ull << b;
    }
    out[w] = lo;
    tmp[w] = eq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t left = need;
    for (int w = 0; w < W && left > 0; ++w) {
      uint64_t eq = tmp[w];
      while (eq && left > 0) {
        const int b = __ffsll((unsigned long long)eq) - 1;
        eq &= eq - 1;
        out[w] |= 1ull << b;
        --left;
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_alg1(int k, int W, const uint64_t *__restrict__ vols,
                                                   const int32_t *__restrict__ n_ld, uint64_t seed,
                                                   uint64_t *Vu, uint64_t *pu, uint64_t *pt,
                                                   uint64_t *nw, uint64_t *po, uint64_t *tmp,
                                                   uint64_t *keys, uint64_t *pj,
                                                   int64_t *vsize, int32_t *order) {
  __shared__ int64_t sh[kThreads / 64 + 2];
  __shared__ uint32_t hist[256];
  // |V_j| and the density order
  for (int j = 0; j < k; ++j) {
    const int64_t c = popcount_set(vols + (size_t)j * W, W, sh);
    if (threadIdx.x == 0) vsize[j] = c;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += kThreads) {
    auto dens = [&](int i) {
      return (vsize[i] > 0 && n_ld[i] > 0) ? fmin(1.0, (double)n_ld[i] / (double)vsize[i]) : -1.0;
    };
    const double dj = dens(j);
    int r = 0;
    for (int i = 0; i < k; ++i) {
      const double di = dens(i);
      r += (di > dj) || (di == dj && i < j);
    }
    order[r] = j;
  }
  for (int w = threadIdx.x; w < W; w += kThreads) {
    Vu[w] = 0;
    pu[w] = 0;
  }
  for (size_t e = threadIdx.x; e < (size_t)k * W; e += kThreads) pj[e] = 0;
  __syncthreads();
  const uint64_t s0 = sm64(seed);
  for (int r = 0; r < k; ++r) {
    const int j = order[r];
    const int64_t vj = vsize[j];
    if (vj <= 0 || n_ld[j] <= 0) continue;     // uniform across the block
    const uint64_t *V = vols + (size_t)j * W;
    const int64_t nVu = popcount_set(Vu, W, sh);
    const int64_t npu = popcount_set(pu, W, sh);
    int64_t thin = target_count(n_ld[j], vj, nVu);
    if (thin > npu) thin = npu;
    select_smallest(pu, npu, thin, W, sm64(s0 ^ (uint64_t)(2 * r)), pt, keys, tmp, sh, hist);
    for (int w = threadIdx.x; w < W; w += kThreads) nw[w] = V[w] & ~Vu[w];
    __syncthreads();
    const int64_t nnew = popcount_set(nw, W, sh);
    const int64_t cnt = target_count(n_ld[j], vj, nnew);
    select_smallest(nw, nnew, cnt, W, sm64(s0 ^ (uint64_t)(2 * r + 1)), po, keys, tmp, sh, hist);
    uint64_t *P = pj + (size_t)j * W;
    for (int w = threadIdx.x; w < W; w += kThreads) {
      P[w] = (pt[w] & V[w]) | po[w];
      pu[w] = pt[w] | po[w];
      Vu[w] |= V[w];
    }
    __syncthreads();
  }
}

// Union of the p_j, then prefix counts of its words (exclusive) and |P|.
__global__ void k_union(int k, int W, const uint64_t *__restrict__ pj, uint64_t *__restrict__ uni) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  uint64_t u = 0;
  for (int j = 0; j < k; ++j) u |= pj[(size_t)j * W + w];
  uni[w] = u;
}

__global__ __launch_bounds__(kThreads) void k_scan_words(int W, const uint64_t *__restrict__ uni,
                                                         int64_t *__restrict__ offs, int64_t *total) {
  __shared__ int64_t part[kThreads];
  const int per = (W + kThreads - 1) / kThreads;
  const int w0 = threadIdx.x * per;
  int64_t s = 0;
  for (int w = w0; w < w0 + per && w < W; ++w) s += __popcll(uni[w]);
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int i = 0; i < kThreads; ++i) {
      const int64_t v = part[i];
      part[i] = acc;
      acc += v;
    }
    *total = acc;
  }
  __syncthreads();
  int64_t acc = part[threadIdx.x];
  for (int w = w0; w < w0 + per && w < W; ++w) {
    offs[w] = acc;
    acc += __popcll(uni[w]);
  }
}

// P[offs[w] + rank of bit] = voxel index.
__global__ void k_compact(int W, const uint64_t *__restrict__ uni, const int64_t *__restrict__ offs,
                          int64_t *__restrict__ P) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  uint64_t word = uni[w];
  int64_t o = offs[w];
  while (word) {
    const int b = __ffsll((unsigned long long)word) - 1;
    word &= word - 1;
    P[o++] = (int64_t)w * 64 + b;
  }
}

// masks[j][i / 64] bit i % 64 = (P[i] in p_j), for i < nP; one thread per (j, word).
__global__ void k_masks(int k, int W, int WP, const uint64_t *__restrict__ pj,
                        const int64_t *__restrict__ P, const int64_t *__restrict__ nP,
                        uint64_t *__restrict__ masks, int ldm) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * WP) return;
  const int j = (int)(e / WP), wi = (int)(e % WP);
  const int64_t n = *nP;
  uint64_t m = 0;
  for (int b = 0; b < 64; ++b) {
    const int64_t i = (int64_t)wi * 64 + b;
    if (i >= n) break;
    const int64_t v = P[i];
    if ((pj[(size_t)j * W + (v >> 6)] >> (v & 63)) & 1ull) m |= 1ull << b;
  }
  masks[(size_t)j * ldm + wi] = m;
}

// Low-dose band: bit v of plan j where lo <= d_j(v) < hi (d from the FP64 product).
__global__ void k_band_bits(const double *__restrict__ d, int ldd, int n_vox, int k, double lo,
                            double hi, uint64_t *__restrict__ bits, int W) {
  // one thread per (plan, word)
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * W) return;
  const int j = (int)(e / W), w = (int)(e % W);
  uint64_t m = 0;
  for (int b = 0; b < 64; ++b) {
    const int v = w * 64 + b;
    if (v >= n_vox) break;
    const double x = d[(size_t)v * ldd + j];
    if (x >= lo && x < hi) m |= 1ull << b;
  }
  bits[(size_t)j * W + w] = m;
}

}  // namespace

hipError_t alg1_select(hipStream_t s, int k, int64_t n_vox, const uint64_t *vols, const int32_t *n_ld,
                       uint64_t seed, Alg1Work &wk, int64_t *P, int64_t *nP, uint64_t *masks, int ldm) {
  const int W = (int)((n_vox + 63) / 64);
  hipLaunchKernelGGL(k_alg1, dim3(1), dim3(kThreads), 0, s, k, W, vols, n_ld, seed, wk.Vu, wk.pu,
                     wk.pt, wk.nw, wk.po, wk.tmp, wk.keys, wk.pj, wk.vsize, wk.order);
  hipLaunchKernelGGL(k_union, dim3((W + 255) / 256), dim3(256), 0, s, k, W, wk.pj, wk.uni);
  hipLaunchKernelGGL(k_scan_words, dim3(1), dim3(kThreads), 0, s, W, wk.uni, wk.offs, nP);
  hipLaunchKernelGGL(k_compact, dim3((W + 255) / 256), dim3(256), 0, s, W, wk.uni, wk.offs, P);
  const int WP = W;   // masks sized for the largest possible |P| = n_vox
  const int64_t tot = (int64_t)k * WP;
  hipLaunchKernelGGL(k_masks, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, k, W, WP, wk.pj,
                     P, nP, masks, ldm);
  return hipGetLastError();
}

hipError_t band_bits(hipStream_t s, const double *d, int ldd, int n_vox, int k, double lo, double hi,
                     uint64_t *bits) {
  const int W = (n_vox + 63) / 64;
  const int64_t tot = (int64_t)k * W;
  hipLaunchKernelGGL(k_band_bits, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, d, ldd,
                     n_vox, k, lo, hi, bits, W);
  return hipGetLastError();
}

}  // namespace ladmm
