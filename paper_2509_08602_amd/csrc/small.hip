// Setup and small-side kernels of the batched ADMM (FP64 unless noted).
//
// Setup (Sec. 2.B, 3.C): scaling of the dose matrix into the point block of A,
// row normalisation E and BOT column scaling beta, assembly of the Schur
// complement S = A_s A_s' + I, its blocked Cholesky factor and the inverse of
// that factor.  Per iteration: the right-hand side of Eq. (partial_elimination),
// the updates of the sector variables and of the m_A-row copy (z2, y2), and the
// per-plan statistics of the stopping test.
//
// Iterate representation.  Every ADMM iterate satisfies z = Pi(z + y), with Pi
// the projection of its block (clip to [0, u] for x1, min(., b) for x2), so the
// device stores only q = z + y; then z = Pi(q) and y = q - Pi(q).  With this,
// the z- and y-steps of Eq. (admm) collapse to q' = z + (x - (z - y)) - ... and
// are written out where they are used below.
#include "kernels.h"

#include <math.h>

#include <algorithm>

namespace ladmm {

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
__global__ void k_scale_dose(const double *__restrict__ phi, int N, int n_t,
                             const double *__restrict__ sig, const double *__restrict__ inv_thr,
                             double *__restrict__ Dt, int Np, int ntp) {
  const size_t total = (size_t)Np * ntp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / ntp), t = (int)(e % ntp);
    Dt[e] = (p < N && t < n_t) ? sig[p] * phi[(size_t)p * n_t + t] * inv_thr[p] : 0.0;
  }
}

// The smallest index of a dose entry that is negative or not finite, into
// *first (which the caller sets to UINT64_MAX); unchanged if there is none.
__global__ void k_check_dose(const double *__restrict__ phi, size_t n, unsigned long long *first) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const double v = phi[e];
    if (!(v >= 0.0) || !isfinite(v)) atomicMin(first, (unsigned long long)e);
  }
}

hipError_t check_dose(hipStream_t s, const double *phi, size_t n, unsigned long long *first) {
  hipLaunchKernelGGL(k_check_dose, dim3(4096), dim3(256), 0, s, phi, n, first);
  return hipGetLastError();
}

hipError_t scale_dose(hipStream_t s, const double *phi, int N, int n_t, const double *sig,
                      const double *inv_thr, double *Dt, int Np, int ntp) {
  hipLaunchKernelGGL(k_scale_dose, dim3(4096), dim3(256), 0, s, phi, N, n_t, sig, inv_thr, Dt,
                     Np, ntp);
  return hipGetLastError();
}

template <typename T>
__global__ void k_scale_columns(const double *__restrict__ Dt, const double *__restrict__ E,
                                T *__restrict__ out, int Np, int ntp) {
  const size_t total = (size_t)Np * ntp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    out[e] = (T)(Dt[e] * E[e % ntp]);
}

template <typename T>
hipError_t scale_columns(hipStream_t s, const double *Dt, const double *E, T *out, int Np, int ntp) {
  hipLaunchKernelGGL((k_scale_columns<T>), dim3(4096), dim3(256), 0, s, Dt, E, out, Np, ntp);
  return hipGetLastError();
}
template hipError_t scale_columns<float>(hipStream_t, const double *, const double *, float *, int, int);
template hipError_t scale_columns<double>(hipStream_t, const double *, const double *, double *, int, int);

template <typename T>
__global__ void k_reduce_partials(const T *__restrict__ P, size_t zstride, int nchunk, int rows,
                                  int cols, int ld, double *__restrict__ out, int ldo) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / cols), c = (int)(e % cols);
    double acc = 0.0;
    for (int z = 0; z < nchunk; ++z) acc += (double)P[z * zstride + (size_t)r * ld + c];
    out[(size_t)r * ldo + c] = acc;
  }
}

template <typename T>
hipError_t reduce_partials(hipStream_t s, const T *P, size_t zstride, int nchunk, int rows,
                           int cols, int ld, double *out, int ldo) {
  hipLaunchKernelGGL((k_reduce_partials<T>), dim3(2048), dim3(256), 0, s, P, zstride, nchunk,
                     rows, cols, ld, out, ldo);
  return hipGetLastError();
}
template hipError_t reduce_partials<float>(hipStream_t, const float *, size_t, int, int, int, int, double *, int);
template hipError_t reduce_partials<double>(hipStream_t, const double *, size_t, int, int, int, int, double *, int);

// E: 1 / (2-norm of each row of the unscaled A).  Shot row t holds the dose
// column t (norm^2 = K[t][t]) and one entry -phi_cal/D_T of C_S'; a BOT row
// holds n_sectors ones (Sec. 3.C).
__global__ void k_row_scales(const double *__restrict__ K, int ldk, SmallLayout L, double cs,
                             int row_normalize, double *__restrict__ E) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= L.mAp) return;
  double e = 0.0;
  if (a < L.n_t) {
    e = row_normalize ? 1.0 / sqrt(K[(size_t)a * ldk + a] + cs * cs) : 1.0;
  } else if (a >= L.ntp && a < L.ntp + L.n_iso) {
    e = row_normalize ? 1.0 / sqrt((double)L.S) : 1.0;
  }
  E[a] = e;
}

// S = A_s A_s' + I with A_s = E A B (B: beta on the sector columns), built from
// K = D~' D~ and the Kronecker structure of C_S and T (App. A).
__global__ void k_assemble_schur(const double *__restrict__ K, int ldk, SmallLayout L,
                                 double cs, double beta, const double *__restrict__ E,
                                 double *__restrict__ S) {
  const size_t total = (size_t)L.mAp * L.mAp;
  const double b2 = beta * beta;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / L.mAp), b = (int)(e % L.mAp);
    const bool atop = a < L.n_t, btop = b < L.n_t;
    const bool abot = a >= L.ntp && a < L.ntp + L.n_iso;
    const bool bbot = b >= L.ntp && b < L.ntp + L.n_iso;
    double v = 0.0;
    if (atop && btop) {
      const double sec = (a / L.C == b / L.C) ? b2 * cs * cs : 0.0;
      v = E[a] * E[b] * (K[(size_t)a * ldk + b] + sec);
    } else if (atop && bbot) {
      v = (a / (L.S * L.C) == b - L.ntp) ? -b2 * cs * E[a] * E[b] : 0.0;
    } else if (abot && btop) {
      v = (b / (L.S * L.C) == a - L.ntp) ? -b2 * cs * E[a] * E[b] : 0.0;
    } else if (abot && bbot) {
      v = (a == b) ? b2 * E[a] * E[b] * (double)L.S : 0.0;
    }
    if (a == b) v += 1.0;
    S[e] = v;
  }
}

hipError_t assemble_schur(hipStream_t s, const double *K, int ldk, const SmallLayout &L, double cs,
                          double beta, double /*e_bot*/, int row_normalize, double *E, double *S) {
  hipLaunchKernelGGL(k_row_scales, dim3((L.mAp + 255) / 256), dim3(256), 0, s, K, ldk, L, cs,
                     row_normalize, E);
  hipLaunchKernelGGL(k_assemble_schur, dim3(2048), dim3(256), 0, s, K, ldk, L, cs, beta, E, S);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// blocked Cholesky (lower) and triangular inverse, FP64, block NB = 32
// ---------------------------------------------------------------------------
constexpr int NB = 32;

// Factor the diagonal block at k0 in LDS (unblocked, column by column).
__global__ void k_potrf_diag(double *S, int ld, int k0, int nb, int *info) {
  __shared__ double a[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    a[i][j] = (j <= i) ? S[(size_t)(k0 + i) * ld + k0 + j] : S[(size_t)(k0 + j) * ld + k0 + i];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (tid == 0) {
      const double d = a[j][j];
      if (!(d > 0.0) || !isfinite(d)) {
        *info = 1;
        a[j][j] = 1.0;
      } else {
        a[j][j] = sqrt(d);
      }
    }
    __syncthreads();
    const double piv = a[j][j];
    for (int i = j + 1 + tid; i < nb; i += blockDim.x) a[i][j] /= piv;
    __syncthreads();
    for (int e = tid; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, c = e % nb;
      if (c > j && i >= c) a[i][c] -= a[i][j] * a[c][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    S[(size_t)(k0 + i) * ld + k0 + j] = (j <= i) ? a[i][j] : 0.0;
  }
}

// Rows below the diagonal block: X L_kk' = S_panel (one thread per row).
__global__ void k_trsm_panel(double *S, int ld, int n, int k0, int nb) {
  __shared__ double l[NB][NB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    l[i][j] = S[(size_t)(k0 + i) * ld + k0 + j];
  }
  __syncthreads();
  const int r = k0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double x[NB];
  double *row = S + (size_t)r * ld + k0;
  for (int c = 0; c < nb; ++c) {
    double v = row[c];
    for (int c2 = 0; c2 < c; ++c2) v -= x[c2] * l[c][c2];
    x[c] = v / l[c][c];
  }
  for (int c = 0; c < nb; ++c) row[c] = x[c];
}

// Trailing update of the lower triangle: S[i][j] -= sum_c S[i][k0+c] S[j][k0+c].
__global__ void k_syrk_update(double *S, int ld, int n, int k0, int nb) {
  const int r0 = k0 + nb;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ double pi[64][NB + 1], pj[64][NB + 1];
  const int i0 = r0 + bi * 64, j0 = r0 + bj * 64;
  for (int e = threadIdx.x; e < 64 * nb; e += blockDim.x) {
    const int rr = e / nb, c = e % nb;
    pi[rr][c] = (i0 + rr < n) ? S[(size_t)(i0 + rr) * ld + k0 + c] : 0.0;
    pj[rr][c] = (j0 + rr < n) ? S[(size_t)(j0 + rr) * ld + k0 + c] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int c = 0; c < nb; ++c) {
    double a[4], b[4];
    for (int u = 0; u < 4; ++u) a[u] = pi[ty * 4 + u][c];
    for (int v = 0; v < 4; ++v) b[v] = pj[tx * 4 + v][c];
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
      if (i < n && j < n && j <= i) S[(size_t)i * ld + j] -= acc[u][v];
    }
}

__global__ void k_zero_upper(double *S, int n, int ld) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (j > i) S[(size_t)i * ld + j] = 0.0;
  }
}

hipError_t cholesky(hipStream_t s, double *S, int n, int ld, int *dinfo) {
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = (n - k0 < NB) ? n - k0 : NB;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, S, ld, k0, nb, dinfo);
    const int rest = n - k0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3((rest + 63) / 64), dim3(64), 0, s, S, ld, n, k0, nb);
      const int tiles = (rest + 63) / 64;
      hipLaunchKernelGGL(k_syrk_update, dim3(tiles, tiles), dim3(256), 0, s, S, ld, n, k0, nb);
    }
  }
  hipLaunchKernelGGL(k_zero_upper, dim3(1024), dim3(256), 0, s, S, n, ld);
  return hipGetLastError();
}

__global__ void k_identity(double *X, int n, int ld) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    X[(size_t)i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
}

// Block row k0 of X: X[k0:k0+nb][c] = L_kk^-1 X[k0:k0+nb][c] for c < k0 + nb.
__global__ void k_trsm_rows(const double *L, double *X, int ld, int k0, int nb) {
  __shared__ double l[NB][NB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    l[i][j] = L[(size_t)(k0 + i) * ld + k0 + j];
  }
  __syncthreads();
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k0 + nb) return;
  double x[NB];
  for (int r = 0; r < nb; ++r) {
    double v = X[(size_t)(k0 + r) * ld + c];
    for (int r2 = 0; r2 < r; ++r2) v -= l[r][r2] * x[r2];
    x[r] = v / l[r][r];
  }
  for (int r = 0; r < nb; ++r) X[(size_t)(k0 + r) * ld + c] = x[r];
}

// X[i][c] -= sum_r L[i][k0+r] X[k0+r][c] for i >= k0 + nb, c < k0 + nb.
__global__ void k_trtri_update(const double *L, double *X, int ld, int n, int k0, int nb) {
  __shared__ double li[64][NB + 1], xr[NB][64 + 1];
  const int i0 = k0 + nb + blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int ncol = k0 + nb;
  for (int e = threadIdx.x; e < 64 * nb; e += blockDim.x) {
    const int rr = e / nb, c = e % nb;
    li[rr][c] = (i0 + rr < n) ? L[(size_t)(i0 + rr) * ld + k0 + c] : 0.0;
  }
  for (int e = threadIdx.x; e < nb * 64; e += blockDim.x) {
    const int r = e / 64, cc = e % 64;
    xr[r][cc] = (c0 + cc < ncol) ? X[(size_t)(k0 + r) * ld + c0 + cc] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int r = 0; r < nb; ++r) {
    double a[4], b[4];
    for (int u = 0; u < 4; ++u) a[u] = li[ty * 4 + u][r];
    for (int v = 0; v < 4; ++v) b[v] = xr[r][tx * 4 + v];
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
  }
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ty * 4 + u, c = c0 + tx * 4 + v;
      if (i < n && c < ncol) X[(size_t)i * ld + c] -= acc[u][v];
    }
}

hipError_t tri_inverse(hipStream_t s, const double *L, double *X, int n, int ld) {
  hipLaunchKernelGGL(k_identity, dim3(1024), dim3(256), 0, s, X, n, ld);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = (n - k0 < NB) ? n - k0 : NB;
    hipLaunchKernelGGL(k_trsm_rows, dim3((k0 + nb + 63) / 64), dim3(64), 0, s, L, X, ld, k0, nb);
    const int rest = n - k0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trtri_update, dim3((k0 + nb + 63) / 64, (rest + 63) / 64), dim3(256),
                         0, s, L, X, ld, n, k0, nb);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per iteration: right-hand side, small-side updates, statistics
// ---------------------------------------------------------------------------
// Grid: (ceil(rows / 4), kp / 64), block (64, 4): x = plan column, y = row.

template <typename T>
__global__ void k_rhs(SmallArgs a, const T *__restrict__ P1, size_t zstride, int nchunk,
                      const double *__restrict__ qs, const double *__restrict__ q2,
                      double *__restrict__ r, const double *__restrict__ gref,
                      double *__restrict__ gout, double *__restrict__ rout,
                      const double *__restrict__ rsub, float *__restrict__ r32) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  const SmallLayout &L = a.L;
  if (m >= L.mAp || j >= a.kp) return;
  const int kp = a.kp;
  double out = 0.0;
  if (m < L.n_t) {
    double g = 0.0;
    // the partials are independent loads: keep several in flight
#pragma unroll 8
    for (int z = 0; z < nchunk; ++z) g += (double)P1[z * zstride + (size_t)m * kp + j];
    if (gout != nullptr && a.active[j]) gout[(size_t)m * kp + j] = g;
    if (gref != nullptr) g += gref[(size_t)m * kp + j];
    const int sec = m / L.C;
    const double qsv = qs[(size_t)sec * kp + j];
    const double wsec = 2.0 * fmax(qsv, 0.0) - qsv;       // z1 - y1 of the sector variable
    const double q2v = q2[(size_t)m * kp + j];
    const double w2 = 2.0 * fmin(q2v, 0.0) - q2v;          // z2 - y2 (b = 0 on shot rows)
    out = g + a.gvec[m] * a.invrho[j] - a.beta * a.E[m] * a.cs * wsec - w2;
  } else if (m >= L.ntp && m < L.ntp + L.n_iso) {
    const int i = m - L.ntp;
    double sum = 0.0;
    for (int s = 0; s < L.S; ++s) {
      const double qsv = qs[(size_t)(i * L.S + s) * kp + j];
      sum += 2.0 * fmax(qsv, 0.0) - qsv;
    }
    const double q2v = q2[(size_t)m * kp + j];
    const double w2 = 2.0 * fmin(q2v, a.bbot[(size_t)i * kp + j]) - q2v;
    out = a.beta * a.E[m] * sum - w2;
  }
  const size_t idx = (size_t)m * kp + j;
  r[idx] = out;
  if (rout != nullptr && a.active[j]) rout[idx] = out;
  if (r32 != nullptr) r32[idx] = (float)(out - rsub[idx]);
}

template <typename T>
hipError_t rhs(hipStream_t s, const SmallArgs &a, const T *P1, size_t zstride, int nchunk,
               const double *qs, const double *q2, double *r, const double *gref, double *gout,
               double *rout, const double *rsub, float *r32) {
  hipLaunchKernelGGL((k_rhs<T>), dim3((a.L.mAp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0, s, a, P1,
                     zstride, nchunk, qs, q2, r, gref, gout, rout, rsub, r32);
  return hipGetLastError();
}
template hipError_t rhs<float>(hipStream_t, const SmallArgs &, const float *, size_t, int, const double *, const double *, double *, const double *, double *, double *, const double *, float *);
template hipError_t rhs<double>(hipStream_t, const SmallArgs &, const double *, size_t, int, const double *, const double *, double *, const double *, double *, double *, const double *, float *);

__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

hipError_t to_f32(hipStream_t s, const double *x, float *y, size_t n) {
  hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

template <typename T>
__global__ void k_vreduce(SmallArgs a, const double *__restrict__ P2, size_t zstride, int nchunk,
                          double *__restrict__ v, T *__restrict__ vT) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.mAp || j >= a.kp) return;
  const size_t idx = (size_t)m * a.kp + j;
  double acc = 0.0;
#pragma unroll 8
  for (int z = 0; z < nchunk; ++z) acc += P2[z * zstride + idx];
  v[idx] = acc;
  if (m < a.L.ntp) vT[idx] = (T)acc;
}

template <typename T>
hipError_t vreduce(hipStream_t s, const SmallArgs &a, const double *P2, size_t zstride, int nchunk,
                   double *v, T *vT) {
  hipLaunchKernelGGL((k_vreduce<T>), dim3((a.L.mAp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0, s,
                     a, P2, zstride, nchunk, v, vT);
  return hipGetLastError();
}
template hipError_t vreduce<float>(hipStream_t, const SmallArgs &, const double *, size_t, int, double *, float *);
template hipError_t vreduce<double>(hipStream_t, const SmallArgs &, const double *, size_t, int, double *, double *);

constexpr int kPostRows = 8;   // rows per block of the post kernel (2 per thread row)

__global__ void k_post(SmallArgs a, const double *__restrict__ v, double *__restrict__ qs,
                       double *__restrict__ q2, double *__restrict__ stats) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const SmallLayout &L = a.L;
  const int kp = a.kp;
  const bool valid = j < kp;
  const bool act = valid && a.active[j] != 0;
  double st[kAdmmStats] = {0, 0, 0, 0, 0, 0};
  const int total = L.mAp + L.n_sec;
  for (int rr = threadIdx.y; valid && rr < kPostRows; rr += 4) {
    const int m = blockIdx.x * kPostRows + rr;
    if (m >= total) break;
    double qv, z, qx, qn, bnd;
    const bool sector = m >= L.mAp;
    if (!sector) {
      const bool top = m < L.n_t;
      const bool bot = m >= L.ntp && m < L.ntp + L.n_iso;
      if (!top && !bot) continue;
      bnd = top ? 0.0 : a.bbot[(size_t)(m - L.ntp) * kp + j];
      qv = q2[(size_t)m * kp + j];
      z = fmin(qv, bnd);
      qx = v[(size_t)m * kp + j] + z;                        // x2 + y2 = v + z2
      qn = a.alpha == 1.0 ? qx : qv + a.alpha * (qx - qv);   // over-relaxed
      if (act) q2[(size_t)m * kp + j] = qn;
    } else {
      const int sec = m - L.mAp;
      const int i = sec / L.S;
      double atv = 0.0;                                      // (A_s' v) at this sector
      for (int c = 0; c < L.C; ++c) {
        const int t = sec * L.C + c;
        atv -= a.beta * a.E[t] * a.cs * v[(size_t)t * kp + j];
      }
      const int mb = L.ntp + i;
      atv += a.beta * a.E[mb] * v[(size_t)mb * kp + j];
      qv = qs[(size_t)sec * kp + j];
      z = fmax(qv, 0.0);
      qx = z - atv;                                          // c = 0, u = +inf here
      qn = a.alpha == 1.0 ? qx : qv + a.alpha * (qx - qv);   // over-relaxed
      if (act) qs[(size_t)sec * kp + j] = qn;
      bnd = INFINITY;
    }
    if (stats != nullptr) {
      const double yo = qv - z;
      const double zn = sector ? fmax(qn, 0.0) : fmin(qn, bnd);
      const double yn = qn - zn;
      const double x = qx - yo;
      const double dxz = a.alpha == 1.0 ? yn - yo : x - zn;   // x - z', unrelaxed x
      st[0] += dxz * dxz;
      st[1] += x * x;
      st[2] += zn * zn;
      st[3] += (zn - z) * (zn - z);
      st[4] += yn * yn;
    }
  }
  if (stats == nullptr) return;
  __shared__ double red[4][kAdmmStats][64];
  for (int q = 0; q < kAdmmStats; ++q) red[threadIdx.y][q][threadIdx.x] = st[q];
  __syncthreads();
  if (threadIdx.y == 0 && valid) {
    for (int q = 0; q < kAdmmStats; ++q) {
      const double s = red[0][q][threadIdx.x] + red[1][q][threadIdx.x] + red[2][q][threadIdx.x] +
                       red[3][q][threadIdx.x];
      stats[((size_t)blockIdx.x * kAdmmStats + q) * kp + j] = s;
    }
  }
}

int post_blocks(const SmallLayout &L) { return (L.mAp + L.n_sec + kPostRows - 1) / kPostRows; }

hipError_t post(hipStream_t s, const SmallArgs &a, const double *v, double *qs, double *q2,
                double *stats, int *nblocks_out) {
  const int nb = post_blocks(a.L);
  if (nblocks_out) *nblocks_out = nb;
  hipLaunchKernelGGL(k_post, dim3(nb, (a.kp + 63) / 64), dim3(64, 4), 0, s, a, v, qs, q2, stats);
  return hipGetLastError();
}

template <typename T>
__global__ void k_shot_scaled(SmallArgs a, const double *__restrict__ q2, T *__restrict__ that) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.ntp || j >= a.kp) return;
  const double ir = a.invrho[j];
  double v = 0.0;
  if (m < a.L.n_t && ir > 0.0) v = fmax(q2[(size_t)m * a.kp + j], 0.0) / ir;
  that[(size_t)m * a.kp + j] = (T)v;
}

template <typename T>
hipError_t shot_scaled(hipStream_t s, const SmallArgs &a, const double *q2, T *that) {
  hipLaunchKernelGGL((k_shot_scaled<T>), dim3((a.L.ntp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0, s, a,
                     q2, that);
  return hipGetLastError();
}
template hipError_t shot_scaled<float>(hipStream_t, const SmallArgs &, const double *, float *);
template hipError_t shot_scaled<double>(hipStream_t, const SmallArgs &, const double *, double *);

// need[t][j] = max(0, (D~' z1)_t) D_T / phi_cal: the smallest value of sector
// (i, s) that shot row t = (i, s, c) allows (App. A: phi' x - C_S' x_sec <= 0),
// from the split-K partials of (D^' z1)_t = E_t (D~' z1)_t.
template <typename T>
__global__ void k_cert_need(SmallArgs a, const T *__restrict__ P, size_t zstride, int nchunk,
                            double *__restrict__ need) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.ntp || j >= a.kp) return;
  double v = 0.0;
  if (m < a.L.n_t) {
    double g = 0.0;
#pragma unroll 8
    for (int z = 0; z < nchunk; ++z) g += (double)P[z * zstride + (size_t)m * a.kp + j];
    v = fmax(0.0, g / a.E[m]) / a.cs;
  }
  need[(size_t)m * a.kp + j] = v;
}

template <typename T>
hipError_t cert_need(hipStream_t s, const SmallArgs &a, const T *P, size_t zstride, int nchunk,
                     double *need) {
  hipLaunchKernelGGL((k_cert_need<T>), dim3((a.L.ntp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0, s,
                     a, P, zstride, nchunk, need);
  return hipGetLastError();
}
template hipError_t cert_need<float>(hipStream_t, const SmallArgs &, const float *, size_t, int, double *);
template hipError_t cert_need<double>(hipStream_t, const SmallArgs &, const double *, size_t, int, double *);

template <typename T>
__global__ void k_z_from_q(const T *__restrict__ q, T *__restrict__ z, int Np, int kp, PointTable<T> pt) {
  const size_t total = (size_t)Np * kp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / kp), j = (int)(e % kp);
    T u = pt.utab[(size_t)pt.grp[p] * pt.ldu + j];
    if (pt.mask != nullptr && pt.is_ld[pt.grp[p]]) {
      const uint64_t w = pt.mask[(size_t)j * pt.mask_words + (p >> 6)];
      if (!((w >> (p & 63)) & 1ull)) u = T(0);
    }
    z[e] = fmin(fmax(q[e], T(0)), u);
  }
}

template <typename T>
hipError_t z_from_q(hipStream_t s, const T *q, T *z, int Np, int kp, const PointTable<T> &pt) {
  hipLaunchKernelGGL((k_z_from_q<T>), dim3(2048), dim3(256), 0, s, q, z, Np, kp, pt);
  return hipGetLastError();
}
template hipError_t z_from_q<float>(hipStream_t, const float *, float *, int, int, const PointTable<float> &);
template hipError_t z_from_q<double>(hipStream_t, const double *, double *, int, int, const PointTable<double> &);

__device__ double block_sum(double v, double *sh) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;   // valid in thread 0
}

__device__ double block_max(double v, double *sh) {
  const int tid = threadIdx.x;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (tid == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}

// One block (256 threads) per plan column.
__global__ void k_finalize(FinalArgs a) {
  __shared__ double sh[8];
  const int j = blockIdx.x, tid = threadIdx.x;
  const int kp = a.kp;
  double s6[kAdmmStats];
  for (int q = 0; q < kAdmmStats; ++q) {
    double v = 0.0;
    for (int b = tid; b < a.admm_blocks; b += blockDim.x)
      v += a.admm_stats[((size_t)b * kAdmmStats + q) * kp + j];
    for (int b = tid; b < a.post_blocks; b += blockDim.x)
      v += a.post_stats[((size_t)b * kAdmmStats + q) * kp + j];
    s6[q] = block_sum(v, sh);
  }
  double hinge = 0.0, oar = 0.0;
  for (int b = tid; b < a.obj_blocks; b += blockDim.x) {
    hinge += a.obj_stats[((size_t)b * kObjStats + 0) * kp + j];
    oar = fmax(oar, a.obj_stats[((size_t)b * kObjStats + 1) * kp + j]);
  }
  double tdose = 0.0;   // sum over targets of u d / D (the OAR repair of the upper bound)
  for (int b = tid; b < a.obj_blocks; b += blockDim.x)
    tdose += a.obj_stats[((size_t)b * kObjStats + 2) * kp + j];
  hinge = block_sum(hinge, sh);
  oar = block_max(oar, sh);
  tdose = block_sum(tdose, sh);
  // beam-on time: tau_i = (phi_cal / D_T) max_s sum_c t_isc, t = E rho max(q2, 0)
  const double ir = a.invrho[j];
  const double rho = ir > 0.0 ? 1.0 / ir : 0.0;
  double bot = 0.0;
  for (int i = tid; i < a.L.n_iso; i += blockDim.x) {
    double best = 0.0;
    for (int s = 0; s < a.L.S; ++s) {
      double sec = 0.0;
      for (int c = 0; c < a.L.C; ++c) {
        const int t = (i * a.L.S + s) * a.L.C + c;
        sec += a.E[t] * rho * fmax(a.q2[(size_t)t * kp + j], 0.0);
      }
      best = fmax(best, sec);
    }
    bot += a.cs * best;
  }
  bot = block_sum(bot, sh);
  // Certificate: the dual point x = (clip(z1), smallest sector values) needs
  // per isocentre i the sum over sectors of the largest collimator value of
  // need; theta = min(1, min_i w_BOT / that sum) keeps every BOT row feasible,
  // and L = -c'(theta x) = -theta c'z1 (c is zero on the sector block).
  double ratio = INFINITY;
  if (a.need != nullptr) {
    const double wb = a.wbot[j];
    for (int i = tid; i < a.L.n_iso; i += blockDim.x) {
      double sum = 0.0;
      for (int s = 0; s < a.L.S; ++s) {
        double best = 0.0;
        for (int c = 0; c < a.L.C; ++c)
          best = fmax(best, a.need[(size_t)((i * a.L.S + s) * a.L.C + c) * kp + j]);
        sum += best;
      }
      if (sum > 0.0) ratio = fmin(ratio, wb / sum);
    }
    for (int o = 32; o > 0; o >>= 1) ratio = fmin(ratio, __shfl_xor(ratio, o));
    if ((tid & 63) == 0) sh[tid >> 6] = ratio;
    __syncthreads();
    if (tid == 0)
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) ratio = fmin(ratio, sh[w]);
    __syncthreads();
  }
  if (tid == 0) {
    const double F = hinge + a.wbot[j] * bot;
    const double cz = s6[5];
    double *o = a.out + (size_t)j * kFinal;
    o[0] = F;
    o[1] = cz;
    o[2] = fabs(F + cz) / fmax(F, 1e-300);
    o[3] = sqrt(s6[0]) / fmax(fmax(sqrt(s6[1]), sqrt(s6[2])), 1e-300);
    o[4] = sqrt(s6[3]) / fmax(sqrt(s6[4]), 1e-300);
    o[5] = oar;
    o[6] = bot;
    o[7] = hinge;
    if (a.need != nullptr) {
      const double theta = fmin(1.0, ratio);
      const double L = -theta * cz;
      // OAR-feasible shot times t / r scale every dose by 1 / r: only the
      // target hinges grow, each by at most (1 - 1/r) u d / D
      const double U = oar > 1.0 ? F + (1.0 - 1.0 / oar) * tdose : F;
      o[8] = L;
      o[9] = (U - L) / fmax(U, 1e-300);
    } else {
      o[8] = NAN;
      o[9] = NAN;
    }
  }
}

hipError_t finalize(hipStream_t s, const FinalArgs &a) {
  hipLaunchKernelGGL(k_finalize, dim3(a.kp), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void k_extract_t(SmallArgs a, const double *__restrict__ q2, double *__restrict__ t, int k) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= k * a.L.n_t) return;
  const int j = idx / a.L.n_t, tt = idx % a.L.n_t;
  const double ir = a.invrho[j];
  t[idx] = ir > 0.0 ? a.E[tt] / ir * fmax(q2[(size_t)tt * a.kp + j], 0.0) : 0.0;
}

hipError_t extract_t(hipStream_t s, const SmallArgs &a, const double *q2, double *t, int k) {
  const int n = k * a.L.n_t;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_extract_t, dim3((n + 255) / 256), dim3(256), 0, s, a, q2, t, k);
  return hipGetLastError();
}

__global__ void k_shot_times_matrix(SmallArgs a, const double *__restrict__ q2, double *__restrict__ out) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.ntp || j >= a.kp) return;
  const double ir = a.invrho[j];
  double v = 0.0;
  if (m < a.L.n_t && ir > 0.0) v = a.E[m] / ir * fmax(q2[(size_t)m * a.kp + j], 0.0);
  out[(size_t)m * a.kp + j] = v;
}

hipError_t shot_times_matrix(hipStream_t s, const SmallArgs &a, const double *q2, double *out) {
  hipLaunchKernelGGL(k_shot_times_matrix, dim3((a.L.ntp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0,
                     s, a, q2, out);
  return hipGetLastError();
}

// Step-size switch on the small rows (z2 = min(q2, b): b = 0 on shot rows,
// E_bot w_BOT on BOT rows) and the sector variables (z = max(qs, 0)).
__global__ void k_rescale_small(SmallArgs a, double *__restrict__ q2, double *__restrict__ qs,
                                double *__restrict__ invrho, const double *__restrict__ fac) {
  const int kp = a.kp;
  const size_t rows = (size_t)a.L.mAp + a.L.n_sec;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < rows * kp;
       e += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / kp), j = (int)(e % kp);
    const double f = fac[j];
    if (f == 1.0) continue;
    if (m < a.L.mAp) {
      const bool bot = m >= a.L.ntp && m < a.L.ntp + a.L.n_iso;
      const double bound = bot ? a.bbot[(size_t)(m - a.L.ntp) * kp + j] : 0.0;
      const double v = q2[e], z = fmin(v, bound);
      q2[e] = z + (v - z) * f;
      if (m == 0) invrho[j] *= f;
    } else {
      const size_t i = e - (size_t)a.L.mAp * kp;
      const double v = qs[i], z = fmax(v, 0.0);
      qs[i] = z + (v - z) * f;
    }
  }
}

hipError_t rescale_small(hipStream_t s, const SmallArgs &a, double *q2, double *qs, double *invrho,
                         const double *fac) {
  hipLaunchKernelGGL(k_rescale_small, dim3(512), dim3(256), 0, s, a, q2, qs, invrho, fac);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// state conversion between q and the (z, y) pair of the oracle's variables
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_export_points(const T *__restrict__ q, int ldq, PointTable<T> pt, int N, int k,
                                double *__restrict__ z, double *__restrict__ y) {
  const size_t total = (size_t)N * k;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / k), j = (int)(e % k);
    const T qv = q[(size_t)p * ldq + j];
    T u = pt.utab[(size_t)pt.grp[p] * pt.ldu + j];
    if (pt.mask != nullptr && pt.is_ld[pt.grp[p]]) {
      const uint64_t w = pt.mask[(size_t)j * pt.mask_words + (p >> 6)];
      if (!((w >> (p & 63)) & 1ull)) u = T(0);
    }
    const T zz = fmin(fmax(qv, T(0)), u);
    z[e] = (double)zz;
    y[e] = (double)qv - (double)zz;
  }
}

template <typename T>
hipError_t export_points(hipStream_t s, const T *q, int ldq, const PointTable<T> &pt, int N, int k,
                         double *z, double *y) {
  hipLaunchKernelGGL((k_export_points<T>), dim3(1024), dim3(256), 0, s, q, ldq, pt, N, k, z, y);
  return hipGetLastError();
}

template <typename T>
__global__ void k_import_points(T *__restrict__ q, int ldq, int N, int k, const double *__restrict__ z,
                                const double *__restrict__ y) {
  const size_t total = (size_t)N * k;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / k), j = (int)(e % k);
    q[(size_t)p * ldq + j] = (T)(z[e] + y[e]);
  }
}

template <typename T>
hipError_t import_points(hipStream_t s, T *q, int ldq, int N, int k, const double *z, const double *y) {
  hipLaunchKernelGGL((k_import_points<T>), dim3(1024), dim3(256), 0, s, q, ldq, N, k, z, y);
  return hipGetLastError();
}
template hipError_t export_points<float>(hipStream_t, const float *, int, const PointTable<float> &, int, int, double *, double *);
template hipError_t export_points<double>(hipStream_t, const double *, int, const PointTable<double> &, int, int, double *, double *);
template hipError_t import_points<float>(hipStream_t, float *, int, int, int, const double *, const double *);
template hipError_t import_points<double>(hipStream_t, double *, int, int, int, const double *, const double *);

// ---------------------------------------------------------------------------
// permutations of plan columns (compaction of the running plans)
// ---------------------------------------------------------------------------
template <typename E>
__global__ void k_gather_cols(const E *__restrict__ in, E *__restrict__ out, size_t rows, int ld,
                              const int *__restrict__ src) {
  const size_t total = rows * (size_t)ld;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / ld;
    out[e] = in[r * ld + src[e % ld]];
  }
}

template <typename E>
__global__ void k_gather_rows(const E *__restrict__ in, E *__restrict__ out, int nrows, size_t len,
                              const int *__restrict__ src) {
  const size_t total = (size_t)nrows * len;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / len;
    out[e] = in[(size_t)src[r] * len + e % len];
  }
}

static unsigned gather_blocks(size_t total) {
  return (unsigned)std::min<size_t>((total + 255) / 256, 8192);
}

hipError_t gather_cols(hipStream_t s, const void *in, void *out, size_t rows, int ld, int bytes,
                       const int *src) {
  const size_t total = rows * (size_t)ld;
  if (total == 0) return hipSuccess;
  const dim3 g(gather_blocks(total)), t(256);
  switch (bytes) {
    case 2: hipLaunchKernelGGL(k_gather_cols<uint16_t>, g, t, 0, s, (const uint16_t *)in, (uint16_t *)out, rows, ld, src); break;
    case 4: hipLaunchKernelGGL(k_gather_cols<uint32_t>, g, t, 0, s, (const uint32_t *)in, (uint32_t *)out, rows, ld, src); break;
    case 8: hipLaunchKernelGGL(k_gather_cols<uint64_t>, g, t, 0, s, (const uint64_t *)in, (uint64_t *)out, rows, ld, src); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t gather_rows(hipStream_t s, const void *in, void *out, int nrows, size_t len, int bytes,
                       const int *src) {
  const size_t total = (size_t)nrows * len;
  if (total == 0) return hipSuccess;
  const dim3 g(gather_blocks(total)), t(256);
  switch (bytes) {
    case 2: hipLaunchKernelGGL(k_gather_rows<uint16_t>, g, t, 0, s, (const uint16_t *)in, (uint16_t *)out, nrows, len, src); break;
    case 4: hipLaunchKernelGGL(k_gather_rows<uint32_t>, g, t, 0, s, (const uint32_t *)in, (uint32_t *)out, nrows, len, src); break;
    case 8: hipLaunchKernelGGL(k_gather_rows<uint64_t>, g, t, 0, s, (const uint64_t *)in, (uint64_t *)out, nrows, len, src); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// a[r][j] = 0 for every row r < rows and column j < ld with flag[j] != 0.
template <typename T>
__global__ void k_zero_columns(T *__restrict__ a, size_t rows, int ld, const int32_t *__restrict__ flag) {
  const size_t total = rows * (size_t)ld;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    if (flag[e % ld]) a[e] = T(0);
}

template <typename T>
hipError_t zero_columns(hipStream_t s, T *a, size_t rows, int ld, const int32_t *flag) {
  if (rows == 0 || ld <= 0) return hipSuccess;
  const size_t total = rows * (size_t)ld;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 2048);
  hipLaunchKernelGGL((k_zero_columns<T>), dim3(blocks), dim3(256), 0, s, a, rows, ld, flag);
  return hipGetLastError();
}
template hipError_t zero_columns<float>(hipStream_t, float *, size_t, int, const int32_t *);
template hipError_t zero_columns<double>(hipStream_t, double *, size_t, int, const int32_t *);

}  // namespace ladmm
