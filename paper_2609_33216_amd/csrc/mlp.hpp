// Rank predictor network (mlp.hip): FP32 parameters on the device, feature
// normalisation on the host.
#pragma once

#include <vector>

#include "common.hpp"
#include "../../include/symhss.h"

namespace symhss {

constexpr int kMlpFeatures = 6;
// largest batch of the allocation-free inference (symhss_predictor_predict_noalloc)
constexpr int kMlpNoAllocSamples = SYMHSS_PREDICT_NOALLOC_MAX;
constexpr int kMlpHidden = 64;
// 6*64+64 + 2*(64*64+64) + 64+1
constexpr int kMlpParams = kMlpFeatures * kMlpHidden + kMlpHidden + 2 * (kMlpHidden * kMlpHidden + kMlpHidden) +
                           kMlpHidden + 1;
static_assert(kMlpParams == SYMHSS_PREDICTOR_WEIGHTS - 2 * kMlpFeatures, "weight vector layout");

class Mlp {
 public:
  Mlp() = default;
  Mlp(const Mlp&) = delete;
  Mlp& operator=(const Mlp&) = delete;
  ~Mlp();
  bool ready() const { return ready_; }
  // host vectors hold the kMlpParams weights followed by the feature means and scales
  void set_params(const float* host, hipStream_t st);
  void get_params(float* host, hipStream_t st) const;
  void train(hipStream_t st, const float* feat, const float* rank, int64_t n, const symhss_train_params& hp,
             float* history);
  void gradient(hipStream_t st, const float* params_host, const float* feat, const float* rank, int64_t n,
                float alpha, float* grad_host, float* loss_host);
  // rank_out[s] = exp(network output) for raw features feat[s * 6 ..]
  void predict(hipStream_t st, const float* feat, int64_t n, float* rank_out);
  // the same with device pointers, activations in `work` (n <= kMlpNoAllocSamples)
  void predict_device(hipStream_t st, const float* feat, int64_t n, float* rank_out, float* work) const;

 private:
  void alloc(int bmax);
  std::vector<float> normalise(const float* feat, int64_t n) const;
  void forward(hipStream_t st, const float* x, int B, float* h1, float* h2, float* h3, float* y) const;
  void loss_grad(hipStream_t st, int B, int n_norm, float alpha);
  float *p_ = nullptr, *g_ = nullptr, *m_ = nullptr, *v_ = nullptr, *ws_ = nullptr;
  int bcap_ = 0;
  double mu_[kMlpFeatures] = {0}, sd_[kMlpFeatures] = {1, 1, 1, 1, 1, 1};
  bool ready_ = false;
};

// Device address of the inference scratch on `device` (which must be
// current), looked up once per device.
float* mlp_scratch_address(int device);

}  // namespace symhss
