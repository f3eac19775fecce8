// Device launchers of the learned RDM propagator (learn.hip), used by the
// C ABI in learn_capi.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

namespace ttns {

enum GemmEpi : int {
  EPI_STORE = 0,  // C = A B
  EPI_BIAS_TANH,  // C = tanh(A B + bias)
  EPI_BIAS_RESID, // C = A B + bias + R
  EPI_TANH_BACK,  // C = (A B) * (1 - R^2)
  EPI_ADD,        // C = A B + C
};

// C[m][n] (m < M, n < N) = epi(sum_k A[m][k] B[k][n]) with element strides
struct GemmArgs {
  int M, N, K;
  const float* A;
  int sam, sak;  // A[m][k] = A[m * sam + k * sak]
  const float* B;
  int sbk, sbn;  // B[k][n] = B[k * sbk + n * sbn]
  float* C;
  int ldc;       // C[m][n] = C[m * ldc + n]
  int epi;
  const float* bias;
  const float* R;  // residual (EPI_BIAS_RESID) or activation (EPI_TANH_BACK)
  int ldr;
};

hipError_t learn_gemm(const GemmArgs& g, hipStream_t s);
hipError_t learn_windows(const int* samples, const float* traj, int T, const float* cond, int ne, int window,
                         int nc, float* X, float* Y, int B, const float* noise, int skip, hipStream_t s);
hipError_t learn_loss(const float* P, const float* Y, int n, float* G, float* partial, int nb, float* loss,
                      hipStream_t s);
hipError_t learn_colsum(const float* G, int M, int N, float* db, hipStream_t s);
hipError_t learn_adam(float* p, const float* g, float* m, float* v, long long n, int* step, float lr,
                      hipStream_t s);
hipError_t learn_rollout_init(const float* init, const float* cond, int B, int ne, int window, int nc, int skip,
                              float* X, hipStream_t s);
hipError_t learn_rollout_post(const float* P, float* X, int B, int ne, int n, int window, int nc, int skip, int in,
                              float* out, int n_steps, int step, hipStream_t s);
hipError_t learn_trace_distance(const float* a, const float* b, int count, int n, float* dist, hipStream_t s);
hipError_t learn_judge(const float* dist, int B, int T, float tol, int* accept, float* worst, hipStream_t s);
hipError_t learn_propagate(const float* src, int stride, const int* samples, const float* U, int n, int B,
                           float* out, hipStream_t s);
hipError_t learn_encode(const double* rdm, long long count, int n, float* out, hipStream_t s);
hipError_t learn_select(const float* pred, const float* ref, const int* accept, int B, long long per, float* out,
                        hipStream_t s);

// Records msg as the calling thread's last error (shared with ttns.h) and
// returns code.
int set_error(int code, const std::string& msg);

constexpr int kLossBlocks = 64;  // partial sums of the loss reduction

}  // namespace ttns
