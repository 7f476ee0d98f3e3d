// Rank predictor: a 6 -> 64 -> 64 -> 64 -> 1 ReLU network in FP32 that maps
// box features to log(ID rank), trained on ranks the solver measures.  The
// paper argues for sizes fixed before the factorisation runs (Section 4.3);
// the predictor supplies them per box.
//
// Kernels: a dense layer forward (one thread per sample and output), the
// asymmetric squared loss on log-rank (under-prediction weighted by alpha)
// and its derivative, the two backward products of a layer (weights: one
// thread per weight summing over the batch in FP64; inputs: one thread per
// sample and input with the ReLU mask), and Adam.  Parameters are one flat
// vector: W1 (64 x 6, row-major), b1, W2 (64 x 64), b2, W3, b3, W4 (1 x 64), b4.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <random>

#include "mlp.hpp"

namespace symhss {

namespace {

constexpr int kIn[4] = {kMlpFeatures, kMlpHidden, kMlpHidden, kMlpHidden};
constexpr int kOut[4] = {kMlpHidden, kMlpHidden, kMlpHidden, 1};

int w_off(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += kIn[i] * kOut[i] + kOut[i];
  return o;
}

__global__ void k_dense_fwd(const float* __restrict__ W, const float* __restrict__ b, const float* __restrict__ X,
                            float* __restrict__ Y, int B, int nin, int nout, int relu) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * nout) return;
  const int s = e / nout, o = e - s * nout;
  float z = b[o];
  const float* w = W + (long)o * nin;
  const float* x = X + (long)s * nin;
  for (int i = 0; i < nin; ++i) z = fmaf(w[i], x[i], z);
  Y[e] = relu ? fmaxf(z, 0.0f) : z;
}

// dz[s] = (2/n) c r, r = yhat - t, c = alpha (r < 0) or 1; loss = (1/n) sum c r^2.
// One workgroup; the loss is summed in FP64 in a fixed order.
__global__ void k_loss(const float* __restrict__ yhat, const float* __restrict__ t, int B, int n_norm,
                       float alpha, float* __restrict__ dz, float* __restrict__ loss) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int s = threadIdx.x; s < B; s += blockDim.x) {
    const float r = yhat[s] - t[s];
    const float c = r < 0.0f ? alpha : 1.0f;
    dz[s] = 2.0f * c * r / (float)n_norm;
    acc += (double)c * (double)r * (double)r;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(part[0] / n_norm);
}

// gW[o, i] = sum_s dZ[s, o] X[s, i]; gb[o] = sum_s dZ[s, o] (threads nin*nout + nout).
__global__ void k_dense_bwd_w(const float* __restrict__ X, const float* __restrict__ dZ, float* __restrict__ gW,
                              float* __restrict__ gb, int B, int nin, int nout) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nin * nout) {
    const int o = e / nin, i = e - o * nin;
    double a = 0.0;
    for (int s = 0; s < B; ++s) a += (double)dZ[(long)s * nout + o] * (double)X[(long)s * nin + i];
    gW[e] = (float)a;
  } else if (e < nin * nout + nout) {
    const int o = e - nin * nout;
    double a = 0.0;
    for (int s = 0; s < B; ++s) a += (double)dZ[(long)s * nout + o];
    gb[o] = (float)a;
  }
}

// dX[s, i] = [X[s, i] > 0] sum_o dZ[s, o] W[o, i]   (X: the ReLU output feeding the layer)
__global__ void k_dense_bwd_x(const float* __restrict__ W, const float* __restrict__ dZ,
                              const float* __restrict__ X, float* __restrict__ dX, int B, int nin, int nout) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * nin) return;
  const int s = e / nin, i = e - s * nin;
  float a = 0.0f;
  if (X[e] > 0.0f) {
    for (int o = 0; o < nout; ++o) a = fmaf(dZ[(long)s * nout + o], W[(long)o * nin + i], a);
  }
  dX[e] = a;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// gather a mini-batch: xb[s] = x[perm[s]], tb[s] = t[perm[s]]
__global__ void k_gather(const float* __restrict__ x, const float* __restrict__ t, const int* __restrict__ perm,
                         int B, float* __restrict__ xb, float* __restrict__ tb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * kMlpFeatures) return;
  const int s = e / kMlpFeatures, f = e - s * kMlpFeatures;
  const int src = perm[s];
  xb[e] = x[(long)src * kMlpFeatures + f];
  if (f == 0) tb[s] = t[src];
}

inline int blocks(long n) { return (int)((n + 255) / 256); }

struct FeatureNorm {
  double mu[kMlpFeatures], sd[kMlpFeatures];
};

// x[s, f] = (feat[s, f] - mu_f) / sd_f, formed in FP64 and rounded once (as
// the host-side normalisation).
__global__ void k_normalise(const float* __restrict__ feat, int n, FeatureNorm nm, float* __restrict__ x) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kMlpFeatures) return;
  const int f = e % kMlpFeatures;
  x[e] = (float)(((double)feat[e] - nm.mu[f]) / nm.sd[f]);
}

// rank[s] = exp(y[s]) in FP64, rounded once.
__global__ void k_exp_rank(const float* __restrict__ y, int n, float* __restrict__ rank) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) rank[s] = (float)exp((double)y[s]);
}

std::mutex g_scratch_mu;
float* g_scratch_ptr[64] = {nullptr};

}  // namespace

// Allocation-free inference: per sample the normalised input, the three
// hidden layers and the output, for at most kMlpNoAllocSamples samples
// (6.5 MB).  Each device holds one copy, shared by every context on it.  Host
// code never uses this name as an address: kernels get the pointer that
// mlp_scratch_address looked up for the device.
constexpr int kInferFloats = kMlpFeatures + 3 * kMlpHidden + 1;
static __device__ __align__(256) float scratch[(size_t)kMlpNoAllocSamples * kInferFloats];

float* mlp_scratch_address(int device) {
  if (device < 0 || device >= 64) throw std::invalid_argument("device index out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != device) throw std::logic_error("scratch lookup with another device current");
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw std::runtime_error("hipGetSymbolAddress returned no address for the inference scratch");
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  return g_scratch_ptr[device];
}

// ---------------------------------------------------------------- Mlp
Mlp::~Mlp() {
  for (float* q : {p_, g_, m_, v_, ws_}) if (q) (void)hipFree(q);
}

void Mlp::alloc(int bmax) {
  if (!p_) {
    HIPCHK(hipMalloc(&p_, kMlpParams * sizeof(float)));
    HIPCHK(hipMalloc(&g_, kMlpParams * sizeof(float)));
    HIPCHK(hipMalloc(&m_, kMlpParams * sizeof(float)));
    HIPCHK(hipMalloc(&v_, kMlpParams * sizeof(float)));
  }
  if (bmax > bcap_) {
    if (ws_) (void)hipFree(ws_);
    ws_ = nullptr;
    // x, t, h1, h2, h3, yhat, dz (B x 64 twice), loss
    const size_t per = kMlpFeatures + 1 + 3 * kMlpHidden + 1 + 2 * kMlpHidden;
    HIPCHK(hipMalloc(&ws_, ((size_t)bmax * per + 64) * sizeof(float)));
    bcap_ = bmax;
  }
}

void Mlp::set_params(const float* host, hipStream_t st) {
  alloc(0);
  HIPCHK(hipMemcpyAsync(p_, host, kMlpParams * sizeof(float), hipMemcpyHostToDevice, st));
  for (int f = 0; f < kMlpFeatures; ++f) {
    mu_[f] = host[kMlpParams + f];
    sd_[f] = host[kMlpParams + kMlpFeatures + f];
    if (!(sd_[f] > 0) || !std::isfinite(sd_[f]) || !std::isfinite(mu_[f]))
      throw std::invalid_argument("predictor normalisation must be finite with positive scales");
  }
  HIPCHK(hipStreamSynchronize(st));
  ready_ = true;
}

void Mlp::get_params(float* host, hipStream_t st) const {
  if (!ready_) throw std::logic_error("predictor has no weights");
  HIPCHK(hipMemcpyAsync(host, p_, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int f = 0; f < kMlpFeatures; ++f) {
    host[kMlpParams + f] = (float)mu_[f];
    host[kMlpParams + kMlpFeatures + f] = (float)sd_[f];
  }
}

std::vector<float> Mlp::normalise(const float* feat, int64_t n) const {
  std::vector<float> x((size_t)n * kMlpFeatures);
  for (int64_t s = 0; s < n; ++s)
    for (int f = 0; f < kMlpFeatures; ++f) {
      const double v = feat[s * kMlpFeatures + f];
      if (!std::isfinite(v)) throw std::invalid_argument("non-finite feature");
      x[s * kMlpFeatures + f] = (float)((v - mu_[f]) / sd_[f]);
    }
  return x;
}

// Workspace layout for a batch of B.
struct MlpWs {
  float *x, *t, *h1, *h2, *h3, *y, *dz, *dz2, *loss;
};
static MlpWs ws_layout(float* w, int B) {
  MlpWs r;
  r.x = w;
  r.t = r.x + (size_t)B * kMlpFeatures;
  r.h1 = r.t + B;
  r.h2 = r.h1 + (size_t)B * kMlpHidden;
  r.h3 = r.h2 + (size_t)B * kMlpHidden;
  r.y = r.h3 + (size_t)B * kMlpHidden;
  r.dz = r.y + B;
  r.dz2 = r.dz + (size_t)B * kMlpHidden;
  r.loss = r.dz2 + (size_t)B * kMlpHidden;
  return r;
}

void Mlp::forward(hipStream_t st, const float* x, int B, float* h1, float* h2, float* h3, float* y) const {
  const float* P = p_;
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks((long)B * kMlpHidden)), dim3(256), 0, st, P + w_off(0),
                     P + w_off(0) + kIn[0] * kOut[0], x, h1, B, kIn[0], kOut[0], 1);
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks((long)B * kMlpHidden)), dim3(256), 0, st, P + w_off(1),
                     P + w_off(1) + kIn[1] * kOut[1], h1, h2, B, kIn[1], kOut[1], 1);
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks((long)B * kMlpHidden)), dim3(256), 0, st, P + w_off(2),
                     P + w_off(2) + kIn[2] * kOut[2], h2, h3, B, kIn[2], kOut[2], 1);
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks(B)), dim3(256), 0, st, P + w_off(3), P + w_off(3) + kIn[3] * kOut[3],
                     h3, y, B, kIn[3], kOut[3], 0);
  HIPCHK(hipGetLastError());
}

// loss and gradient of the batch held in workspace x / t (g_ receives the gradient)
void Mlp::loss_grad(hipStream_t st, int B, int n_norm, float alpha) {
  MlpWs w = ws_layout(ws_, B);
  forward(st, w.x, B, w.h1, w.h2, w.h3, w.y);
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, w.y, w.t, B, n_norm, alpha, w.dz, w.loss);
  // layer 4 (64 -> 1): dZ = dz (B x 1)
  const float* acts[4] = {w.x, w.h1, w.h2, w.h3};
  float* dzc = w.dz;   // gradient at the current layer's output (B x nout)
  float* dzn = w.dz2;  // gradient at its input
  for (int l = 3; l >= 0; --l) {
    float* gW = g_ + w_off(l);
    float* gb = gW + kIn[l] * kOut[l];
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks(kIn[l] * kOut[l] + kOut[l])), dim3(256), 0, st, acts[l], dzc, gW,
                       gb, B, kIn[l], kOut[l]);
    if (l > 0) {
      hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks((long)B * kIn[l])), dim3(256), 0, st, p_ + w_off(l), dzc,
                         acts[l], dzn, B, kIn[l], kOut[l]);
      std::swap(dzc, dzn);
    }
  }
  HIPCHK(hipGetLastError());
}

void Mlp::gradient(hipStream_t st, const float* params_host, const float* feat, const float* rank, int64_t n,
                   float alpha, float* grad_host, float* loss_host) {
  if (n < 1 || n > (1 << 24)) throw std::invalid_argument("sample count out of range");
  set_params(params_host, st);
  alloc((int)n);
  std::vector<float> x = normalise(feat, n);
  std::vector<float> t(n);
  for (int64_t s = 0; s < n; ++s) {
    if (!(rank[s] >= 1.0f) || !std::isfinite(rank[s])) throw std::invalid_argument("ranks must be >= 1");
    t[s] = std::log(rank[s]);
  }
  MlpWs w = ws_layout(ws_, (int)n);
  HIPCHK(hipMemcpyAsync(w.x, x.data(), x.size() * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.t, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice, st));
  loss_grad(st, (int)n, (int)n, alpha);
  HIPCHK(hipMemcpyAsync(grad_host, g_, kMlpParams * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(loss_host, w.loss, sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

void Mlp::train(hipStream_t st, const float* feat, const float* rank, int64_t n, const symhss_train_params& hp,
                float* history) {
  if (n < 1 || n > (1 << 24)) throw std::invalid_argument("sample count out of range");
  if (hp.epochs < 1 || hp.batch < 1 || !(hp.lr > 0) || !(hp.alpha >= 1))
    throw std::invalid_argument("epochs, batch >= 1, lr > 0, alpha >= 1 required");
  // feature normalisation from the training set
  for (int f = 0; f < kMlpFeatures; ++f) {
    double s = 0, q = 0;
    for (int64_t i = 0; i < n; ++i) s += feat[i * kMlpFeatures + f];
    const double mu = s / n;
    for (int64_t i = 0; i < n; ++i) {
      const double d = feat[i * kMlpFeatures + f] - mu;
      q += d * d;
    }
    const double sd = std::sqrt(q / n);
    mu_[f] = mu;
    sd_[f] = sd > 0 ? sd : 1.0;
  }
  std::vector<float> x = normalise(feat, n);
  std::vector<float> t(n);
  for (int64_t s = 0; s < n; ++s) {
    if (!(rank[s] >= 1.0f) || !std::isfinite(rank[s])) throw std::invalid_argument("ranks must be >= 1");
    t[s] = std::log(rank[s]);
  }
  // He-normal initialisation, zero biases
  std::mt19937_64 rng(hp.seed);
  std::normal_distribution<float> nd(0.0f, 1.0f);
  std::vector<float> p(kMlpParams + 2 * kMlpFeatures, 0.0f);
  for (int l = 0; l < 4; ++l) {
    const float sc = std::sqrt(2.0f / kIn[l]);
    for (int e = 0; e < kIn[l] * kOut[l]; ++e) p[w_off(l) + e] = sc * nd(rng);
  }
  for (int f = 0; f < kMlpFeatures; ++f) {
    p[kMlpParams + f] = (float)mu_[f];
    p[kMlpParams + kMlpFeatures + f] = (float)sd_[f];
  }
  set_params(p.data(), st);
  const int B = (int)std::min<int64_t>(hp.batch, n);
  alloc(B);
  float *dx = nullptr, *dt = nullptr, *dloss = nullptr;
  int* dperm = nullptr;
  const int steps_per_epoch = (int)((n + B - 1) / B);
  HIPCHK(hipMalloc(&dx, x.size() * sizeof(float)));
  HIPCHK(hipMalloc(&dt, t.size() * sizeof(float)));
  HIPCHK(hipMalloc(&dperm, n * sizeof(int)));
  HIPCHK(hipMalloc(&dloss, (size_t)hp.epochs * steps_per_epoch * sizeof(float)));
  struct Free {
    void* q[4];
    ~Free() { for (void* v : q) if (v) (void)hipFree(v); }
  } fr{{dx, dt, dperm, dloss}};
  HIPCHK(hipMemcpyAsync(dx, x.data(), x.size() * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dt, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(m_, 0, kMlpParams * sizeof(float), st));
  HIPCHK(hipMemsetAsync(v_, 0, kMlpParams * sizeof(float), st));
  std::vector<int> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  int tstep = 0;
  MlpWs w = ws_layout(ws_, B);
  for (int ep = 0; ep < hp.epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    HIPCHK(hipMemcpyAsync(dperm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // perm is host memory reused next epoch
    for (int k = 0; k < steps_per_epoch; ++k) {
      const int b0 = k * B;
      const int bs = (int)std::min<int64_t>(B, n - b0);
      w = ws_layout(ws_, bs);
      hipLaunchKernelGGL(k_gather, dim3(blocks((long)bs * kMlpFeatures)), dim3(256), 0, st, dx, dt, dperm + b0, bs,
                         w.x, w.t);
      loss_grad(st, bs, bs, hp.alpha);
      ++tstep;
      const float c1 = 1.0f - std::pow(b1, (float)tstep), c2 = 1.0f - std::pow(b2, (float)tstep);
      hipLaunchKernelGGL(k_adam, dim3(blocks(kMlpParams)), dim3(256), 0, st, p_, g_, m_, v_, kMlpParams, hp.lr, b1,
                         b2, eps, c1, c2);
      HIPCHK(hipMemcpyAsync(dloss + (size_t)ep * steps_per_epoch + k, w.loss, sizeof(float),
                            hipMemcpyDeviceToDevice, st));
    }
  }
  HIPCHK(hipGetLastError());
  std::vector<float> lh((size_t)hp.epochs * steps_per_epoch);
  HIPCHK(hipMemcpyAsync(lh.data(), dloss, lh.size() * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (history)
    for (int ep = 0; ep < hp.epochs; ++ep) {
      double s = 0;
      for (int k = 0; k < steps_per_epoch; ++k) s += lh[(size_t)ep * steps_per_epoch + k];
      history[ep] = (float)(s / steps_per_epoch);
    }
}

// Queued on st only: nothing is allocated, copied to the host or waited for.
// work: the device's inference scratch (mlp_scratch_address).  Features are
// not checked (that would need a wait): a non-finite one gives a non-finite
// rank.
void Mlp::predict_device(hipStream_t st, const float* feat, int64_t n, float* rank_out, float* work) const {
  if (!ready_) throw std::logic_error("predictor has no weights");
  if (n < 0 || n > kMlpNoAllocSamples)
    throw std::invalid_argument("sample count must be in 0.." + std::to_string(kMlpNoAllocSamples));
  if (n == 0) return;
  if (!feat || !rank_out || !work) throw std::invalid_argument("null device pointer");
  const int B = (int)n;
  float* x = work;
  float* h1 = x + (size_t)B * kMlpFeatures;
  float* h2 = h1 + (size_t)B * kMlpHidden;
  float* h3 = h2 + (size_t)B * kMlpHidden;
  float* y = h3 + (size_t)B * kMlpHidden;
  FeatureNorm nm;
  for (int f = 0; f < kMlpFeatures; ++f) {
    nm.mu[f] = mu_[f];
    nm.sd[f] = sd_[f];
  }
  hipLaunchKernelGGL(k_normalise, dim3(blocks((long)B * kMlpFeatures)), dim3(256), 0, st, feat, B, nm, x);
  forward(st, x, B, h1, h2, h3, y);
  hipLaunchKernelGGL(k_exp_rank, dim3(blocks(B)), dim3(256), 0, st, y, B, rank_out);
  HIPCHK(hipGetLastError());
}

void Mlp::predict(hipStream_t st, const float* feat, int64_t n, float* rank_out) {
  if (!ready_) throw std::logic_error("predictor has no weights");
  if (n <= 0) return;
  if (n > (1 << 24)) throw std::invalid_argument("sample count out of range");
  alloc((int)n);
  std::vector<float> x = normalise(feat, n);
  MlpWs w = ws_layout(ws_, (int)n);
  HIPCHK(hipMemcpyAsync(w.x, x.data(), x.size() * sizeof(float), hipMemcpyHostToDevice, st));
  forward(st, w.x, (int)n, w.h1, w.h2, w.h3, w.y);
  std::vector<float> y(n);
  HIPCHK(hipMemcpyAsync(y.data(), w.y, n * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int64_t s = 0; s < n; ++s) rank_out[s] = std::exp(y[s]);
}

}  // namespace symhss
