// Host side of the learned RDM propagator: workspace layout, the launch
// sequences of training (forward, loss, backward, Adam), rollout and
// judging, and the C-ABI entry points of include/ttnn.h.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "learn_internal.h"
#include "ttnn.h"

using namespace ttns;

#define LCHK(x)                                                                          \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return set_error(TTNS_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct ttnn_net {
  ttnn_config cfg{};
  int ne = 0, in0 = 0;
  std::vector<int> sizes;                  // layer widths, input first
  std::vector<int64_t> w_off, b_off;       // flat offsets of W and b per layer
  int64_t s_off = -1;                      // flat offset of the skip matrix W_s
  int64_t n_params = 0;
  hipStream_t stream = nullptr;
  // device buffers inside the caller's workspace
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;
  int* step = nullptr;
  int* samples = nullptr;
  float *X = nullptr, *Y = nullptr, *Pout = nullptr, *dOut = nullptr;
  std::vector<float*> H;
  float* dH[2] = {nullptr, nullptr};
  float *lpart = nullptr, *loss = nullptr;
  float* Rres = nullptr;  // residual base enc(U rho_t U^dagger) of every row
  // training data (caller's device arrays)
  const float* traj = nullptr;
  const float* cond = nullptr;
  const float* prop = nullptr;  // per-set free propagators, or null
  int n_sets = 0, n_times = 0;
};

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int check_config(const ttnn_config* c) {
  if (!c) return set_error(TTNS_EINVAL, "ttnn: null config");
  if (c->n_levels < 1 || c->n_levels > 8) return set_error(TTNS_EINVAL, "ttnn: n_levels must be in [1, 8]");
  if (c->window < 1 || c->n_cond < 0 || c->hidden < 1 || c->layers < 1 || c->layers > 8 || c->max_batch < 1 ||
      c->skip < 0 || c->skip > 1)
    return set_error(TTNS_EINVAL,
                     "ttnn: window, hidden, max_batch >= 1, n_cond >= 0, layers in [1, 8], skip 0 or 1");
  const int64_t ne = (int64_t)c->n_levels * c->n_levels;
  const int64_t in0 = c->window * ne + c->n_cond + (c->skip ? c->n_cond * ne : 0);
  if (in0 > (1 << 20) || c->hidden > (1 << 16) || (int64_t)c->max_batch * std::max<int64_t>(in0, c->hidden) > (1ll << 30))
    return set_error(TTNS_EINVAL, "ttnn: network too large");
  return TTNS_OK;
}

// Layout of the workspace (offsets from its base); `net` receives the
// pointers when base is not null.
size_t layout(const ttnn_config& c, char* base, ttnn_net* net) {
  const int ne = c.n_levels * c.n_levels;
  const int in0 = c.window * ne + c.n_cond + (c.skip ? c.n_cond * ne : 0);
  std::vector<int> sizes{in0};
  for (int l = 0; l < c.layers; ++l) sizes.push_back(c.hidden);
  sizes.push_back(ne);
  int64_t np = 0;
  std::vector<int64_t> wo, bo;
  for (size_t l = 0; l + 1 < sizes.size(); ++l) {
    wo.push_back(np);
    np += (int64_t)sizes[l] * sizes[l + 1];
    bo.push_back(np);
    np += sizes[l + 1];
  }
  int64_t so = -1;
  if (c.skip) {
    so = np;
    np += (int64_t)ne * in0;
  }
  const size_t B = c.max_batch;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return base ? base + o : nullptr;
  };
  char* p = take(np * 4);
  char* g = take(np * 4);
  char* mo = take(np * 4);
  char* vo = take(np * 4);
  char* st = take(4);
  char* sm = take(2 * B * 4);
  char* x = take(B * in0 * 4);
  char* y = take(B * ne * 4);
  char* po = take(B * ne * 4);
  char* dO = take(B * ne * 4);
  std::vector<char*> h;
  for (int l = 0; l < c.layers; ++l) h.push_back(take(B * c.hidden * 4));
  char* d0 = take(B * c.hidden * 4);
  char* d1 = take(B * c.hidden * 4);
  char* lp = take(kLossBlocks * 4);
  char* ls = take(4);
  char* rr = take(B * ne * 4);
  if (net) {
    net->cfg = c;
    net->ne = ne;
    net->in0 = in0;
    net->sizes = sizes;
    net->w_off = wo;
    net->b_off = bo;
    net->s_off = so;
    net->n_params = np;
    net->P = (float*)p;
    net->G = (float*)g;
    net->Mo = (float*)mo;
    net->Vo = (float*)vo;
    net->step = (int*)st;
    net->samples = (int*)sm;
    net->X = (float*)x;
    net->Y = (float*)y;
    net->Pout = (float*)po;
    net->dOut = (float*)dO;
    net->H.clear();
    for (char* q : h) net->H.push_back((float*)q);
    net->dH[0] = (float*)d0;
    net->dH[1] = (float*)d1;
    net->lpart = (float*)lp;
    net->loss = (float*)ls;
    net->Rres = (float*)rr;
  }
  return off;
}

GemmArgs gemm(int M, int N, int K, const float* A, int sam, int sak, const float* Bm, int sbk, int sbn, float* C,
              int ldc, int epi = EPI_STORE, const float* bias = nullptr, const float* R = nullptr, int ldr = 0) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.sam = sam;
  g.sak = sak;
  g.B = Bm;
  g.sbk = sbk;
  g.sbn = sbn;
  g.C = C;
  g.ldc = ldc;
  g.epi = epi;
  g.bias = bias;
  g.R = R;
  g.ldr = ldr;
  return g;
}

// Forward pass of B rows of X into H[.] and Pout; the output adds the
// residual base: Rres when the rows have free propagators, else the last
// RDM of each row's window.
int forward(ttnn_net& n, int B, bool propagated) {
  const ttnn_config& c = n.cfg;
  const float* a = n.X;
  int lda = n.in0;
  for (int l = 0; l < c.layers; ++l) {
    const int in = n.sizes[l], out = n.sizes[l + 1];
    LCHK(learn_gemm(gemm(B, out, in, a, lda, 1, n.P + n.w_off[l], 1, in, n.H[l], c.hidden, EPI_BIAS_TANH,
                         n.P + n.b_off[l]),
                    n.stream));
    a = n.H[l];
    lda = c.hidden;
  }
  const int L = c.layers;
  const float* base = propagated ? n.Rres : n.X + (size_t)(c.window - 1) * n.ne;
  const int ldb = propagated ? n.ne : n.in0;
  LCHK(learn_gemm(gemm(B, n.ne, c.hidden, a, lda, 1, n.P + n.w_off[L], 1, c.hidden, n.Pout, n.ne, EPI_BIAS_RESID,
                       n.P + n.b_off[L], base, ldb),
                  n.stream));
  if (c.skip)  // Pout += X W_s^T
    LCHK(learn_gemm(gemm(B, n.ne, n.in0, n.X, n.in0, 1, n.P + n.s_off, 1, n.in0, n.Pout, n.ne, EPI_ADD), n.stream));
  return TTNS_OK;
}

// Loss of Pout against Y and the gradient of every parameter into G.
int backward(ttnn_net& n, int B) {
  const ttnn_config& c = n.cfg;
  LCHK(learn_loss(n.Pout, n.Y, B * n.ne, n.dOut, n.lpart, kLossBlocks, n.loss, n.stream));
  if (c.skip)  // dW_s = dOut^T X
    LCHK(learn_gemm(gemm(n.ne, n.in0, B, n.dOut, 1, n.ne, n.X, n.in0, 1, n.G + n.s_off, n.in0), n.stream));
  const float* g = n.dOut;
  int ldg = n.ne;
  for (int l = c.layers; l >= 0; --l) {
    const int in = n.sizes[l], out = n.sizes[l + 1];
    const float* a = l == 0 ? n.X : n.H[l - 1];
    const int lda = l == 0 ? n.in0 : c.hidden;
    // dW = g^T a (out x in), db = column sums of g
    LCHK(learn_gemm(gemm(out, in, B, g, 1, ldg, a, lda, 1, n.G + n.w_off[l], in), n.stream));
    LCHK(learn_colsum(g, B, out, n.G + n.b_off[l], n.stream));
    if (l > 0) {
      float* ng = n.dH[l % 2];
      LCHK(learn_gemm(gemm(B, in, out, g, ldg, 1, n.P + n.w_off[l], in, 1, ng, c.hidden, EPI_TANH_BACK, nullptr,
                           n.H[l - 1], c.hidden),
                      n.stream));
      g = ng;
      ldg = c.hidden;
    }
  }
  return TTNS_OK;
}

int load_batch(ttnn_net& n, const int32_t* host_samples, int batch, const float* dev_noise = nullptr) {
  if (!n.traj) return set_error(TTNS_EINVAL, "ttnn: no training data (ttnn_set_data)");
  if (!host_samples || batch < 1 || batch > n.cfg.max_batch)
    return set_error(TTNS_EINVAL, "ttnn: batch must be in [1, max_batch]");
  for (int b = 0; b < batch; ++b) {
    const int s = host_samples[2 * b], t = host_samples[2 * b + 1];
    if (s < 0 || s >= n.n_sets || t < n.cfg.window - 1 || t >= n.n_times - 1)
      return set_error(TTNS_EINVAL, "ttnn: sample " + std::to_string(b) + " out of range");
  }
  LCHK(hipMemcpyAsync(n.samples, host_samples, (size_t)batch * 2 * sizeof(int32_t), hipMemcpyHostToDevice,
                      n.stream));
  LCHK(learn_windows(n.samples, n.traj, n.n_times, n.cond, n.ne, n.cfg.window, n.cfg.n_cond, n.X, n.Y, batch,
                     dev_noise, n.cfg.skip, n.stream));
  if (n.prop)
    LCHK(learn_propagate(n.X + (size_t)(n.cfg.window - 1) * n.ne, n.in0, n.samples, n.prop, n.cfg.n_levels, batch,
                         n.Rres, n.stream));
  return TTNS_OK;
}

}  // namespace

extern "C" {

int ttnn_param_count(const ttnn_config* cfg, int64_t* count) {
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!count) return set_error(TTNS_EINVAL, "ttnn_param_count: null output");
  ttnn_net tmp;
  layout(*cfg, nullptr, &tmp);
  *count = tmp.n_params;
  return TTNS_OK;
}

int ttnn_workspace_size(const ttnn_config* cfg, size_t* bytes) {
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!bytes) return set_error(TTNS_EINVAL, "ttnn_workspace_size: null output");
  *bytes = layout(*cfg, nullptr, nullptr);
  return TTNS_OK;
}

int ttnn_build(const ttnn_config* cfg, const float* host_params, void* dev_ws, size_t ws_bytes, void* hip_stream,
               ttnn_net** out) {
  int rc = check_config(cfg);
  if (rc) return rc;
  if (!host_params || !dev_ws || !out) return set_error(TTNS_EINVAL, "ttnn_build: null argument");
  if ((uintptr_t)dev_ws % 256) return set_error(TTNS_EINVAL, "ttnn_build: workspace must be 256-byte aligned");
  const size_t need = layout(*cfg, nullptr, nullptr);
  if (ws_bytes < need) return set_error(TTNS_ENOMEM, "ttnn_build: workspace too small: need " + std::to_string(need));
  ttnn_net* n = new ttnn_net;
  layout(*cfg, (char*)dev_ws, n);
  n->stream = (hipStream_t)hip_stream;
  rc = ttnn_set_params(n, host_params);
  if (rc) {
    delete n;
    return rc;
  }
  *out = n;
  return TTNS_OK;
}

int ttnn_conditioning(const ttns_star_model* m, float* host_out, int32_t n_out, int32_t* written) {
  if (!m || !host_out || !written || !m->h_el || m->n_levels < 1 || m->n_chains < 0 ||
      (m->n_chains > 0 && (!m->alpha || !m->coupling)))
    return set_error(TTNS_EINVAL, "ttnn_conditioning: bad model");
  const int n = m->n_levels, nc = m->n_chains;
  const int need = n + n * (n - 1) / 2 + nc * (1 + n);
  if (n_out < need) return set_error(TTNS_EINVAL, "ttnn_conditioning: output needs " + std::to_string(need));
  int k = 0;
  for (int j = 0; j < n; ++j) host_out[k++] = (float)m->h_el[j * n + j].re;
  for (int j = 0; j < n; ++j)
    for (int l = j + 1; l < n; ++l) host_out[k++] = (float)m->h_el[j * n + l].re;
  for (int i = 0; i < nc; ++i) host_out[k++] = (float)m->alpha[i];
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < n; ++j) host_out[k++] = (float)m->coupling[(size_t)i * n * n + j * n + j].re;
  *written = k;
  return TTNS_OK;
}

int ttnn_propagator(const ttns_star_model* m, double dt, float* host_out, int32_t n_out) {
  if (!m || !m->h_el || m->n_levels < 1 || m->n_levels > 8 || !host_out || !std::isfinite(dt))
    return set_error(TTNS_EINVAL, "ttnn_propagator: bad arguments");
  const int n = m->n_levels;
  if (n_out < 2 * n * n) return set_error(TTNS_EINVAL, "ttnn_propagator: output needs 2 n^2 floats");
  // exp(-i H dt): scale to 1-norm <= 1/2, Taylor to 24 terms, square back
  typedef std::complex<double> z;
  std::vector<z> A(n * n), E(n * n, 0.0), term(n * n), tmp(n * n);
  double nrm = 0.0;
  for (int j = 0; j < n; ++j) {
    double col = 0.0;
    for (int i = 0; i < n; ++i) col += std::abs(z(m->h_el[i * n + j].re, m->h_el[i * n + j].im)) * std::fabs(dt);
    nrm = std::max(nrm, col);
  }
  int sq = 0;
  while (nrm > 0.5 && sq < 60) {
    nrm *= 0.5;
    ++sq;
  }
  const double scale = std::ldexp(dt, -sq);
  for (int i = 0; i < n * n; ++i) A[i] = z(0.0, -1.0) * z(m->h_el[i].re, m->h_el[i].im) * scale;
  auto mul = [&](const std::vector<z>& X, const std::vector<z>& Y, std::vector<z>& out) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        z acc = 0.0;
        for (int l = 0; l < n; ++l) acc += X[i * n + l] * Y[l * n + j];
        out[i * n + j] = acc;
      }
  };
  for (int i = 0; i < n; ++i) E[i * n + i] = 1.0;
  term = E;
  for (int k = 1; k <= 24; ++k) {
    mul(term, A, tmp);
    for (int i = 0; i < n * n; ++i) {
      term[i] = tmp[i] / (double)k;
      E[i] += term[i];
    }
  }
  for (int q = 0; q < sq; ++q) {
    mul(E, E, tmp);
    E = tmp;
  }
  for (int i = 0; i < n * n; ++i) {
    host_out[2 * i] = (float)E[i].real();
    host_out[2 * i + 1] = (float)E[i].imag();
  }
  return TTNS_OK;
}

int ttnn_encode(ttnn_net* n, const double* dev_rdm, int64_t count, float* dev_out) {
  if (!n || count < 0 || (count > 0 && (!dev_rdm || !dev_out))) return set_error(TTNS_EINVAL, "ttnn_encode: bad arguments");
  if (count == 0) return TTNS_OK;
  LCHK(learn_encode(dev_rdm, count, n->cfg.n_levels, dev_out, n->stream));
  return TTNS_OK;
}

int ttnn_set_data(ttnn_net* n, const float* dev_traj, const float* dev_cond, const float* dev_prop,
                  int32_t n_sets, int32_t n_times) {
  if (!n || !dev_traj || (n->cfg.n_cond > 0 && !dev_cond) || n_sets < 1 || n_times < n->cfg.window + 1)
    return set_error(TTNS_EINVAL, "ttnn_set_data: need n_sets >= 1 and n_times >= window + 1");
  n->traj = dev_traj;
  n->cond = dev_cond;
  n->prop = dev_prop;
  n->n_sets = n_sets;
  n->n_times = n_times;
  return TTNS_OK;
}

int ttnn_gradients(ttnn_net* n, const int32_t* host_samples, int32_t batch, float* host_loss, float* host_grad) {
  if (!n || !host_loss) return set_error(TTNS_EINVAL, "ttnn_gradients: null argument");
  int rc = load_batch(*n, host_samples, batch);
  if (!rc) rc = forward(*n, batch, n->prop != nullptr);
  if (!rc) rc = backward(*n, batch);
  if (rc) return rc;
  if (host_grad)
    LCHK(hipMemcpyAsync(host_grad, n->G, (size_t)n->n_params * 4, hipMemcpyDeviceToHost, n->stream));
  LCHK(hipMemcpyAsync(host_loss, n->loss, 4, hipMemcpyDeviceToHost, n->stream));
  LCHK(hipStreamSynchronize(n->stream));
  return TTNS_OK;
}

int ttnn_train_step(ttnn_net* n, const int32_t* host_samples, int32_t batch, float lr, const float* dev_noise) {
  if (!n || !(lr > 0)) return set_error(TTNS_EINVAL, "ttnn_train_step: bad arguments");
  int rc = load_batch(*n, host_samples, batch, dev_noise);
  if (!rc) rc = forward(*n, batch, n->prop != nullptr);
  if (!rc) rc = backward(*n, batch);
  if (rc) return rc;
  // the next call's sample copy is ordered after these launches on the stream
  LCHK(learn_adam(n->P, n->G, n->Mo, n->Vo, n->n_params, n->step, lr, n->stream));
  return TTNS_OK;
}

int ttnn_last_loss(ttnn_net* n, float* host_loss) {
  if (!n || !host_loss) return set_error(TTNS_EINVAL, "ttnn_last_loss: null argument");
  LCHK(hipMemcpyAsync(host_loss, n->loss, 4, hipMemcpyDeviceToHost, n->stream));
  LCHK(hipStreamSynchronize(n->stream));
  return TTNS_OK;
}

int ttnn_get_params(ttnn_net* n, float* host_out) {
  if (!n || !host_out) return set_error(TTNS_EINVAL, "ttnn_get_params: null argument");
  LCHK(hipMemcpyAsync(host_out, n->P, (size_t)n->n_params * 4, hipMemcpyDeviceToHost, n->stream));
  LCHK(hipStreamSynchronize(n->stream));
  return TTNS_OK;
}

int ttnn_set_params(ttnn_net* n, const float* host_in) {
  if (!n || !host_in) return set_error(TTNS_EINVAL, "ttnn_set_params: null argument");
  LCHK(hipMemcpyAsync(n->P, host_in, (size_t)n->n_params * 4, hipMemcpyHostToDevice, n->stream));
  LCHK(hipMemsetAsync(n->Mo, 0, (size_t)n->n_params * 4, n->stream));
  LCHK(hipMemsetAsync(n->Vo, 0, (size_t)n->n_params * 4, n->stream));
  LCHK(hipMemsetAsync(n->step, 0, 4, n->stream));
  LCHK(hipMemsetAsync(n->loss, 0, 4, n->stream));
  LCHK(hipStreamSynchronize(n->stream));
  return TTNS_OK;
}

int ttnn_rollout(ttnn_net* n, const float* dev_init, const float* dev_cond, const float* dev_prop, int32_t batch,
                 int32_t n_steps, float* dev_out) {
  if (!n || batch < 1 || batch > n->cfg.max_batch || n_steps < 0 || !dev_init || !dev_out ||
      (n->cfg.n_cond > 0 && !dev_cond))
    return set_error(TTNS_EINVAL, "ttnn_rollout: bad arguments (batch must be in [1, max_batch])");
  const ttnn_config& c = n->cfg;
  LCHK(learn_rollout_init(dev_init, dev_cond, batch, n->ne, c.window, c.n_cond, c.skip, n->X, n->stream));
  for (int s = 0; s < n_steps; ++s) {
    if (dev_prop)
      LCHK(learn_propagate(n->X + (size_t)(c.window - 1) * n->ne, n->in0, nullptr, dev_prop, c.n_levels, batch,
                           n->Rres, n->stream));
    int rc = forward(*n, batch, dev_prop != nullptr);
    if (rc) return rc;
    LCHK(learn_rollout_post(n->Pout, n->X, batch, n->ne, c.n_levels, c.window, c.n_cond, c.skip, n->in0, dev_out,
                            n_steps, s, n->stream));
  }
  return TTNS_OK;
}

int ttnn_judge(ttnn_net* n, const float* dev_pred, const float* dev_ref, int32_t batch, int32_t n_steps, float tol,
               float* dev_dist, float* dev_worst, int32_t* dev_accept) {
  if (!n || batch < 1 || n_steps < 1 || !dev_pred || !dev_ref || !dev_dist || !dev_worst || !dev_accept ||
      !(tol >= 0))
    return set_error(TTNS_EINVAL, "ttnn_judge: bad arguments");
  const long long count = (long long)batch * n_steps;
  if (count > (1ll << 31) - 1) return set_error(TTNS_EINVAL, "ttnn_judge: too many matrices");
  LCHK(learn_trace_distance(dev_pred, dev_ref, (int)count, n->cfg.n_levels, dev_dist, n->stream));
  LCHK(learn_judge(dev_dist, batch, n_steps, tol, dev_accept, dev_worst, n->stream));
  return TTNS_OK;
}

int ttnn_select(ttnn_net* n, const float* dev_pred, const float* dev_ref, const int32_t* dev_accept, int32_t batch,
                int32_t n_steps, float* dev_out) {
  if (!n || batch < 1 || n_steps < 0 || !dev_pred || !dev_ref || !dev_accept || !dev_out)
    return set_error(TTNS_EINVAL, "ttnn_select: bad arguments");
  if (n_steps == 0) return TTNS_OK;
  LCHK(learn_select(dev_pred, dev_ref, dev_accept, batch, (long long)n_steps * n->ne, dev_out, n->stream));
  return TTNS_OK;
}

int ttnn_destroy(ttnn_net* n) {
  delete n;
  return TTNS_OK;
}

}  // extern "C"
