// Learned propagator of the electronic reduced density matrix: device code.
//
// A multilayer perceptron maps the last `window` encoded RDMs of a
// trajectory plus the model's conditioning reals to the next RDM (residual
// form: enc(rho_{t+1}) = enc(rho_t) + net(x)).  Training (forward, backward,
// Adam) and batched autoregressive rollouts run here; the full TTNS run of
// the same parameters judges every rollout by the trace distance.
//
// GEMMs use v_mfma_f32_16x16x4_f32 on 64 x 64 output tiles (4 wavefronts,
// 32 x 32 each), K staged through LDS 16 at a time, FP32 accumulation, with
// fused epilogues.  Encoding of an n x n Hermitian RDM into n^2 reals: the
// diagonal, then Re and Im of the upper triangle (j < k, row-major).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "learn_internal.h"

namespace ttns {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ float As[GT][GK + 1];
  __shared__ float Bs[GK][GT + 4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0, 0, 0, 0};
  for (int k0 = 0; k0 < g.K; k0 += GK) {
    for (int e = t; e < GT * GK; e += 256) {
      const int r = e / GK, c = e % GK;
      const int m = m0 + r, k = k0 + c;
      As[r][c] = (m < g.M && k < g.K) ? g.A[(size_t)m * g.sam + (size_t)k * g.sak] : 0.f;
    }
    for (int e = t; e < GT * GK; e += 256) {
      const int r = e / GT, c = e % GT;
      const int k = k0 + r, n = n0 + c;
      Bs[r][c] = (k < g.K && n < g.N) ? g.B[(size_t)k * g.sbk + (size_t)n * g.sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kq = kk + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wm + 16 * i + (lane & 15)][kq];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kq][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][q];
        switch (g.epi) {
          case EPI_BIAS_TANH:
            v = tanhf(v + g.bias[n]);
            break;
          case EPI_BIAS_RESID:
            v = v + g.bias[n] + g.R[(size_t)m * g.ldr + n];
            break;
          case EPI_ADD:
            v = v + g.C[(size_t)m * g.ldc + n];
            break;
          case EPI_TANH_BACK: {
            const float h = g.R[(size_t)m * g.ldr + n];
            v = v * (1.f - h * h);
            break;
          }
          default:
            break;
        }
        g.C[(size_t)m * g.ldc + n] = v;
      }
}

// X[b] = [traj[s][t-window+1 .. t] (window x ne) (+ noise[b]), cond[s],
// (skip) cond[s][c] * x_last[e] for (c, e) row-major], Y[b] = traj[s][t+1]
__global__ void k_windows(const int* samples, const float* traj, int T, const float* cond, int ne,
                          int window, int nc, float* X, float* Y, int B, const float* noise, int skip) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const int s = samples[2 * b], t = samples[2 * b + 1];
  const int wn = window * ne;
  const int in = wn + nc + (skip ? nc * ne : 0);
  const float* tr = traj + (size_t)s * T * ne;
  const float* nz = noise ? noise + (size_t)b * wn : nullptr;
  for (int i = threadIdx.x; i < in; i += blockDim.x) {
    float v;
    if (i < wn) {
      v = tr[(size_t)(t - window + 1) * ne + i];
      if (nz) v += nz[i];
    } else if (i < wn + nc) {
      v = cond[(size_t)s * nc + (i - wn)];
    } else {
      const int c = (i - wn - nc) / ne, e = (i - wn - nc) % ne;
      float last = tr[(size_t)t * ne + e];
      if (nz) last += nz[(window - 1) * ne + e];
      v = cond[(size_t)s * nc + c] * last;
    }
    X[(size_t)b * in + i] = v;
  }
  if (Y)
    for (int i = threadIdx.x; i < ne; i += blockDim.x) Y[(size_t)b * ne + i] = tr[(size_t)(t + 1) * ne + i];
}

// loss = mean (P - Y)^2 (block partials, folded by one thread in order),
// G = 2 (P - Y) / (B ne)
__global__ void k_loss(const float* P, const float* Y, int n, float* G, float* partial) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float d = P[i] - Y[i];
    G[i] = 2.f * d / (float)n;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_fold(const float* partial, int nb, int n, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < nb; ++i) s += partial[i];
    *loss = s / (float)n;
  }
}

// db[n] = sum_m G[m][n]  (one thread per column, m in order)
__global__ void k_colsum(const float* G, int M, int N, float* db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += G[(size_t)m * N + n];
  db[n] = s;
}

// Adam with bias correction; step counter on the device (incremented by the
// last thread of block 0 after use: the next launch sees t + 1)
__global__ void k_adam(float* p, const float* g, float* m, float* v, long long n, const int* step, float lr) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = *step;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  if (i < n) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  }
}
__global__ void k_step_inc(int* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

// Rollout: prediction -> divide by the trace -> output and window shift
// (X rows: [window x ne | cond | (skip) cond x last]); the bilinear block
// is recomputed from the new last RDM.
__global__ void k_rollout_post(const float* P, float* X, int B, int ne, int n, int window, int nc, int skip,
                               int in, float* out, int n_steps, int step) {
  const int b = blockIdx.x;
  if (b >= B) return;
  __shared__ float tr;
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int j = 0; j < n; ++j) s += P[(size_t)b * ne + j];
    tr = s;
  }
  __syncthreads();
  const float inv = 1.f / tr;
  // shift the window left by one RDM (in order: read before write per element)
  float* x = X + (size_t)b * in;
  for (int base = 0; base < (window - 1) * ne; base += blockDim.x) {
    const int i = base + threadIdx.x;
    float v = 0.f;
    if (i < (window - 1) * ne) v = x[i + ne];
    __syncthreads();
    if (i < (window - 1) * ne) x[i] = v;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < ne; i += blockDim.x) {
    const float e = P[(size_t)b * ne + i] * inv;
    x[(window - 1) * ne + i] = e;
    out[((size_t)b * n_steps + step) * ne + i] = e;
  }
  if (skip) {
    __syncthreads();
    const int wn = window * ne;
    for (int i = threadIdx.x; i < nc * ne; i += blockDim.x)
      x[wn + nc + i] = x[wn + i / ne] * x[(window - 1) * ne + i % ne];
  }
}

// Trace distance 1/2 sum |eig(rho - sigma)| of n x n Hermitian matrices
// given in the n^2-real encoding (n <= 8), one thread per pair.  The
// Hermitian difference H = X + iY is embedded as the real symmetric
// [[X, -Y], [Y, X]] (every eigenvalue of H twice) and diagonalised by cyclic
// Jacobi rotations in FP64: t = sgn(th) / (|th| + sqrt(th^2 + 1)),
// th = (a_qq - a_pp) / (2 a_pq), c = 1 / sqrt(1 + t^2), s = t c.
__global__ void k_trace_distance(const float* a, const float* b, int count, int n, float* dist) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= count) return;
  const int ne = n * n, m = n * (n - 1) / 2, N = 2 * n;
  double A[16][16];
  const float* pa = a + (size_t)id * ne;
  const float* pb = b + (size_t)id * ne;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) A[i][j] = 0.0;
  for (int j = 0; j < n; ++j) {
    const double x = (double)pa[j] - (double)pb[j];
    A[j][j] = x;
    A[n + j][n + j] = x;
  }
  int q = 0;
  for (int j = 0; j < n; ++j)
    for (int k = j + 1; k < n; ++k, ++q) {
      const double x = (double)pa[n + q] - (double)pb[n + q];      // Re H_jk
      const double y = (double)pa[n + m + q] - (double)pb[n + m + q];  // Im H_jk
      A[j][k] = A[k][j] = x;
      A[n + j][n + k] = A[n + k][n + j] = x;
      // lower-left block Y (Y_jk = y, Y_kj = -y), upper-right -Y
      A[n + j][k] = y;
      A[n + k][j] = -y;
      A[j][n + k] = -y;
      A[k][n + j] = y;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < N; ++p)
      for (int r = p + 1; r < N; ++r) off += A[p][r] * A[p][r];
    if (off < 1e-28) break;
    for (int p = 0; p < N; ++p)
      for (int r = p + 1; r < N; ++r) {
        const double apr = A[p][r];
        if (fabs(apr) < 1e-300) continue;
        const double th = (A[r][r] - A[p][p]) / (2.0 * apr);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < N; ++k) {
          const double x = A[k][p], y = A[k][r];
          A[k][p] = c * x - s * y;
          A[k][r] = s * x + c * y;
        }
        for (int k = 0; k < N; ++k) {
          const double x = A[p][k], y = A[r][k];
          A[p][k] = c * x - s * y;
          A[r][k] = s * x + c * y;
        }
      }
  }
  double tsum = 0.0;
  for (int j = 0; j < N; ++j) tsum += fabs(A[j][j]);
  dist[id] = (float)(0.25 * tsum);  // each eigenvalue twice, times 1/2
}

// accept[b] = max_t dist[b][t] <= tol; worst[b] = that maximum
__global__ void k_judge(const float* dist, int B, int T, float tol, int* accept, float* worst) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float mx = 0.f;
  for (int t = 0; t < T; ++t) mx = fmaxf(mx, dist[(size_t)b * T + t]);
  worst[b] = mx;
  accept[b] = mx <= tol ? 1 : 0;
}

// X[b] = [init[b] (window x ne), cond[b], (skip) cond[b] x last of init[b]]
__global__ void k_rollout_init(const float* init, const float* cond, int ne, int window, int nc, int skip, float* X) {
  const int b = blockIdx.x;
  const int wn = window * ne;
  const int in = wn + nc + (skip ? nc * ne : 0);
  const float* w = init + (size_t)b * wn;
  const float* c = cond + (size_t)b * nc;
  for (int i = threadIdx.x; i < in; i += blockDim.x) {
    float v;
    if (i < wn) v = w[i];
    else if (i < wn + nc) v = c[i - wn];
    else v = c[(i - wn - nc) / ne] * w[(window - 1) * ne + (i - wn - nc) % ne];
    X[(size_t)b * in + i] = v;
  }
}

// rdm: count x n x n complex (re, im doubles, row-major) -> n^2 reals
__global__ void k_encode(const double* rdm, long long count, int n, float* out) {
  const int ne = n * n, m = n * (n - 1) / 2;
  const long long total = count * ne;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long c = i / ne;
    const int e = (int)(i % ne);
    const double* r = rdm + (size_t)c * ne * 2;
    double v;
    if (e < n) {
      v = r[2 * (e * n + e)];
    } else {
      const int q = e < n + m ? e - n : e - n - m;  // upper-triangle index
      int j = 0, rem = q;
      while (rem >= n - 1 - j) {
        rem -= n - 1 - j;
        ++j;
      }
      const int k = j + 1 + rem;
      v = r[2 * (j * n + k) + (e < n + m ? 0 : 1)];
    }
    out[i] = (float)v;
  }
}

// out[b] = accept[b] ? pred[b] : ref[b], `per` floats per b
__global__ void k_select(const float* pred, const float* ref, const int* accept, int B, long long per, float* out) {
  const long long total = (long long)B * per;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(i / per);
    out[i] = accept[b] ? pred[i] : ref[i];
  }
}

// out[b] = enc(U rho U^dagger), rho = decoded row b of src (row stride
// `stride`, n^2 reals), U = the n x n complex propagator (2 n^2 floats,
// (re, im) row-major) of set samples[2b] (training) or of row b (samples
// null).  One workgroup of 64 threads per row, thread (j, k) = entry jk.
__global__ void k_propagate(const float* src, int stride, const int* samples, const float* U, int n, float* out) {
  const int b = blockIdx.x;
  const int t = threadIdx.x, j = t / n, k = t % n;
  const int ne = n * n, m = n * (n - 1) / 2;
  __shared__ double2 rho[64], u[64], mu[64];
  const int set = samples ? samples[2 * b] : b;
  const float* r = src + (size_t)b * stride;
  const float* uu = U + (size_t)set * 2 * ne;
  const bool on = t < ne;
  // upper-triangle index of (min, max) pair, row-major
  auto q_of = [&](int a, int c) { return a * n - a * (a + 1) / 2 + (c - a - 1); };
  if (on) {
    double2 v;
    if (j == k) v = make_double2(r[j], 0.0);
    else if (j < k) v = make_double2(r[n + q_of(j, k)], r[n + m + q_of(j, k)]);
    else v = make_double2(r[n + q_of(k, j)], -r[n + m + q_of(k, j)]);
    rho[t] = v;
    u[t] = make_double2(uu[2 * t], uu[2 * t + 1]);
  }
  __syncthreads();
  if (on) {  // (U rho)[j][k]
    double2 acc = make_double2(0.0, 0.0);
    for (int l = 0; l < n; ++l) acc = cfma(u[j * n + l], rho[l * n + k], acc);
    mu[t] = acc;
  }
  __syncthreads();
  if (on) {  // (U rho U^dagger)[j][k] = sum_l (U rho)[j][l] conj(U[k][l])
    double2 acc = make_double2(0.0, 0.0);
    for (int l = 0; l < n; ++l) {
      const double2 a = mu[j * n + l], c = u[k * n + l];
      acc.x += a.x * c.x + a.y * c.y;
      acc.y += a.y * c.x - a.x * c.y;
    }
    float* o = out + (size_t)b * ne;
    if (j == k) o[j] = (float)acc.x;
    else if (j < k) {
      o[n + q_of(j, k)] = (float)acc.x;
      o[n + m + q_of(j, k)] = (float)acc.y;
    }
  }
}

// ---------------------------------------------------------------- launchers
hipError_t learn_gemm(const GemmArgs& g, hipStream_t s) {
  const dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}
hipError_t learn_windows(const int* samples, const float* traj, int T, const float* cond, int ne,
                         int window, int nc, float* X, float* Y, int B, const float* noise, int skip,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_windows, dim3(B), dim3(256), 0, s, samples, traj, T, cond, ne, window, nc, X, Y, B, noise,
                     skip);
  return hipGetLastError();
}
hipError_t learn_loss(const float* P, const float* Y, int n, float* G, float* partial, int nb, float* loss,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, P, Y, n, G, partial);
  hipLaunchKernelGGL(k_loss_fold, dim3(1), dim3(64), 0, s, partial, nb, n, loss);
  return hipGetLastError();
}
hipError_t learn_colsum(const float* G, int M, int N, float* db, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, G, M, N, db);
  return hipGetLastError();
}
hipError_t learn_adam(float* p, const float* g, float* m, float* v, long long n, int* step, float lr,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, step, lr);
  return hipGetLastError();
}
hipError_t learn_rollout_post(const float* P, float* X, int B, int ne, int n, int window, int nc, int skip, int in,
                              float* out, int n_steps, int step, hipStream_t s) {
  hipLaunchKernelGGL(k_rollout_post, dim3(B), dim3(256), 0, s, P, X, B, ne, n, window, nc, skip, in, out, n_steps,
                     step);
  return hipGetLastError();
}
hipError_t learn_trace_distance(const float* a, const float* b, int count, int n, float* dist, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_distance, dim3((count + 127) / 128), dim3(128), 0, s, a, b, count, n, dist);
  return hipGetLastError();
}
hipError_t learn_rollout_init(const float* init, const float* cond, int B, int ne, int window, int nc, int skip,
                              float* X, hipStream_t s) {
  hipLaunchKernelGGL(k_rollout_init, dim3(B), dim3(256), 0, s, init, cond, ne, window, nc, skip, X);
  return hipGetLastError();
}
hipError_t learn_propagate(const float* src, int stride, const int* samples, const float* U, int n, int B,
                           float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_propagate, dim3(B), dim3(64), 0, s, src, stride, samples, U, n, out);
  return hipGetLastError();
}
hipError_t learn_encode(const double* rdm, long long count, int n, float* out, hipStream_t s) {
  const long long total = count * n * n;
  const unsigned nb = (unsigned)std::min<long long>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_encode, dim3(nb), dim3(256), 0, s, rdm, count, n, out);
  return hipGetLastError();
}
hipError_t learn_select(const float* pred, const float* ref, const int* accept, int B, long long per, float* out,
                        hipStream_t s) {
  const long long total = (long long)B * per;
  const unsigned nb = (unsigned)std::min<long long>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_select, dim3(nb), dim3(256), 0, s, pred, ref, accept, B, per, out);
  return hipGetLastError();
}
hipError_t learn_judge(const float* dist, int B, int T, float tol, int* accept, float* worst, hipStream_t s) {
  hipLaunchKernelGGL(k_judge, dim3((B + 255) / 256), dim3(256), 0, s, dist, B, T, tol, accept, worst);
  return hipGetLastError();
}

}  // namespace ttns
