// C-ABI of the solver (include/symhss.h): argument checks, the stage
// machine and the mapping of C++ exceptions to status codes.  No exception
// crosses this boundary.
#include <cmath>
#include <new>
#include <stdexcept>
#include <string>

#include "solver.hpp"

struct symhss_ctx {
  symhss::Solver* s = nullptr;
  std::string err;
};

namespace {

thread_local std::string g_create_error;

template <class F>
symhss_status guarded(symhss_ctx* ctx, F&& f) {
  if (!ctx || !ctx->s) return SYMHSS_EINVAL;
  symhss::BudgetScope budget(ctx->s->budget());
  try {
    f(*ctx->s);
    ctx->err.clear();
    return SYMHSS_OK;
  } catch (const std::bad_alloc&) {
    ctx->err = "out of memory";
    return SYMHSS_ENOMEM;
  } catch (const std::invalid_argument& e) {
    ctx->err = e.what();
    return SYMHSS_EINVAL;
  } catch (const std::logic_error& e) {
    ctx->err = e.what();
    if (dynamic_cast<const std::domain_error*>(&e)) return SYMHSS_ESINGULAR;
    return SYMHSS_ESTATE;
  } catch (const std::range_error& e) {
    ctx->err = e.what();
    return SYMHSS_ERANK;
  } catch (const symhss::NotConverged& e) {
    ctx->err = e.what();
    return SYMHSS_ENOTCONV;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return SYMHSS_EDEVICE;
  } catch (...) {
    ctx->err = "unknown error";
    return SYMHSS_EDEVICE;
  }
}

}  // namespace

extern "C" {

symhss_status symhss_create(symhss_ctx** out, int device, void* hip_stream) {
  if (!out) return SYMHSS_EINVAL;
  *out = nullptr;
  int ndev = 0;
  const hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) {
    g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
    return SYMHSS_EDEVICE;
  }
  if (device < 0 || device >= ndev) {
    g_create_error = "device index " + std::to_string(device) + " out of range (" + std::to_string(ndev) + " devices)";
    return SYMHSS_EDEVICE;
  }
  symhss_ctx* c = new (std::nothrow) symhss_ctx();
  if (!c) return SYMHSS_ENOMEM;
  try {
    c->s = new symhss::Solver(device, static_cast<hipStream_t>(hip_stream));
  } catch (const std::exception& ex) {
    g_create_error = ex.what();
    delete c;
    return SYMHSS_EDEVICE;
  }
  *out = c;
  return SYMHSS_OK;
}

void symhss_destroy(symhss_ctx* ctx) {
  if (!ctx) return;
  delete ctx->s;
  delete ctx;
}

const char* symhss_last_error(const symhss_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

void* symhss_stream(symhss_ctx* ctx) { return (ctx && ctx->s) ? static_cast<void*>(ctx->s->stream()) : nullptr; }

symhss_status symhss_assemble(symhss_ctx* ctx, int64_t n, const double* x, const double* dx, const double* ddx,
                              const symhss_medium* medium, const symhss_opts* opts) {
  if (!medium || !opts) return SYMHSS_EINVAL;
  return guarded(ctx, [&](symhss::Solver& s) { s.assemble(n, x, dx, ddx, *medium, *opts); });
}

symhss_status symhss_assemble_batch(symhss_ctx* ctx, int32_t count, const int64_t* n, const double* x,
                                    const double* dx, const double* ddx, const symhss_medium* media,
                                    const symhss_opts* opts) {
  if (!opts || !n || !media || count < 1) return SYMHSS_EINVAL;
  return guarded(ctx, [&](symhss::Solver& s) { s.assemble_batch(count, n, x, dx, ddx, media, *opts); });
}

symhss_status symhss_compress(symhss_ctx* ctx) {
  return guarded(ctx, [&](symhss::Solver& s) { s.compress(); });
}

symhss_status symhss_factor(symhss_ctx* ctx) {
  return guarded(ctx, [&](symhss::Solver& s) { s.factor(); });
}

symhss_status symhss_factor_solve(symhss_ctx* ctx, const symhss_z* b, symhss_z* x, int32_t nrhs, int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) { s.factor_solve(b, x, nrhs, flags); });
}

symhss_status symhss_solve(symhss_ctx* ctx, const symhss_z* b, symhss_z* x, int32_t nrhs, int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) { s.solve(b, x, nrhs, flags); });
}

symhss_status symhss_solve_incident(symhss_ctx* ctx, const symhss_z* uin, const symhss_z* qin, symhss_z* q,
                                    symhss_z* u, int32_t nrhs, int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) { s.solve_incident(uin, qin, q, u, nrhs, flags); });
}

symhss_status symhss_plane_wave(symhss_ctx* ctx, const double* angles, symhss_z* uin, symhss_z* qin,
                                int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) { s.plane_wave_incident(angles, uin, qin, flags); });
}

symhss_status symhss_rhs_plane_wave(symhss_ctx* ctx, double angle, symhss_z* b, int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!b) throw std::invalid_argument("null output");
    s.rhs_plane_wave(angle, b, flags);
  });
}

symhss_status symhss_rhs_plane_wave_batch(symhss_ctx* ctx, const double* angles, symhss_z* b, int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!b || !angles) throw std::invalid_argument("null argument");
    s.rhs_plane_wave_batch(angles, b, flags);
  });
}

symhss_status symhss_eval_entries(symhss_ctx* ctx, int64_t nr, const int64_t* rows, int64_t nc,
                                  const int64_t* cols, symhss_z* out) {
  return guarded(ctx, [&](symhss::Solver& s) { s.eval_entries(nr, rows, nc, cols, out); });
}

symhss_status symhss_eval_bessel(symhss_ctx* ctx, int64_t n, const double* z, double* out) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (n < 0 || (n && (!z || !out))) throw std::invalid_argument("bad arguments");
    for (int64_t i = 0; i < n; ++i)
      if (!(z[i] > 0) || !std::isfinite(z[i])) throw std::invalid_argument("z must be positive and finite");
    s.eval_bessel(n, z, out);
  });
}

symhss_status symhss_matvec_direct(symhss_ctx* ctx, const symhss_z* x, symhss_z* y, int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!x || !y) throw std::invalid_argument("null vector");
    s.matvec_direct(x, y, flags);
  });
}

symhss_status symhss_configure(symhss_ctx* ctx, int32_t option, int64_t value) {
  return guarded(ctx, [&](symhss::Solver& s) { s.configure(option, value); });
}

symhss_status symhss_predictor_train(symhss_ctx* ctx, const float* feat, const float* rank, int64_t n,
                                     const symhss_train_params* hp, float* history) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!feat || !rank || !hp) throw std::invalid_argument("null argument");
    s.predictor().train(s.stream(), feat, rank, n, *hp, history);
  });
}

symhss_status symhss_predictor_load(symhss_ctx* ctx, const float* weights, int64_t count) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!weights || count != SYMHSS_PREDICTOR_WEIGHTS) throw std::invalid_argument("need SYMHSS_PREDICTOR_WEIGHTS floats");
    for (int64_t i = 0; i < count; ++i)
      if (!std::isfinite(weights[i])) throw std::invalid_argument("non-finite weight");
    s.predictor().set_params(weights, s.stream());
  });
}

symhss_status symhss_predictor_get(symhss_ctx* ctx, float* weights, int64_t count) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!weights || count != SYMHSS_PREDICTOR_WEIGHTS) throw std::invalid_argument("need SYMHSS_PREDICTOR_WEIGHTS floats");
    s.predictor().get_params(weights, s.stream());
  });
}

symhss_status symhss_predictor_predict(symhss_ctx* ctx, const float* feat, int64_t n, float* rank_out) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (n < 0 || (n && (!feat || !rank_out))) throw std::invalid_argument("bad arguments");
    s.predictor().predict(s.stream(), feat, n, rank_out);
  });
}

symhss_status symhss_predictor_predict_noalloc(symhss_ctx* ctx, const float* feat, int64_t n, float* rank_out) {
  return guarded(ctx, [&](symhss::Solver& s) {
    s.predictor().predict_device(s.stream(), feat, n, rank_out, s.infer_scratch());
  });
}

symhss_status symhss_predictor_grad(symhss_ctx* ctx, const float* weights, const float* feat, const float* rank,
                                    int64_t n, float alpha, float* grad, float* loss) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!weights || !feat || !rank || !grad || !loss) throw std::invalid_argument("null argument");
    if (!(alpha >= 1.0f)) throw std::invalid_argument("alpha must be >= 1");
    s.predictor().gradient(s.stream(), weights, feat, rank, n, alpha, grad, loss);
  });
}

symhss_status symhss_box_table(symhss_ctx* ctx, int64_t* count, float* feat, int32_t* rank, int32_t* info) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!count) throw std::invalid_argument("null count");
    s.box_table(count, feat, rank, info);
  });
}

symhss_status symhss_hss_matvec(symhss_ctx* ctx, const symhss_z* x, symhss_z* y, int32_t flags) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!x || !y) throw std::invalid_argument("null vector");
    s.hss_matvec(x, y, flags);
  });
}

symhss_status symhss_get_stats(const symhss_ctx* ctx, symhss_stats* out) {
  if (!ctx || !ctx->s || !out) return SYMHSS_EINVAL;
  *out = ctx->s->stats();
  return SYMHSS_OK;
}

symhss_status symhss_box_query(symhss_ctx* ctx, int32_t level, int32_t box, int32_t what, int64_t* count,
                               void* out) {
  return guarded(ctx, [&](symhss::Solver& s) {
    if (!count) throw std::invalid_argument("null count");
    s.box_query(level, box, what, count, out);
  });
}

}  // extern "C"
