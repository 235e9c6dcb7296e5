// C ABI of the learned choice of lambda: features of the data in the KP-SVD
// basis, the optimal-error targets, and the network (mlp.h) that maps the
// features to log10(lambda), with GCV (Section 2.2, eq. (GCVTikSVD), in the
// Kronecker basis of Section 5.1) as the judge of its answer.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "capi_internal.h"
#include "mlp.h"

using namespace kpcg;

// lambda_predict_noalloc's activations (see scratch_address below)
constexpr size_t kNoallocBytes = kpcg::mlp_act_bytes(KP_PREDICT_NOALLOC_MAX_ROWS);
static_assert(kNoallocBytes == KP_PREDICT_NOALLOC_BYTES, "header states the array's size");
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

struct kp_mlp_s {
  Mlp M;
  float* feat1 = nullptr;    // device staging for kp_lambda_learned
  double* pred1 = nullptr;
};

namespace {

constexpr float kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;
constexpr int kMaxBatch = 65536;

size_t model_bytes(int max_batch) {
  return (mlp_layout(max_batch, nullptr, nullptr) + 255) / 256 * 256 + 1024;
}

// lambda_predict_noalloc: the forward activations of up to
// KP_PREDICT_NOALLOC_MAX_ROWS rows in a static device array (each GPU the
// library runs on holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel or copy: it is a host-side
// stand-in, not a device address.  The device address is looked up once per
// device with hipGetSymbolAddress (that device current) and kept: at
// mlp_create, or on the entry point's first call on a device where no model
// was created.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return KP_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) return KP_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KP_OK;
}

int read_loss(const Mlp& M, double* out, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(M.host_loss, M.loss, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *out = *M.host_loss;
  return KP_OK;
}

}  // namespace

extern "C" {

int kp_features(kp_plan_t plan, const float* b, float* features_out, void* stream) {
  if (!plan || !b || !features_out || !aligned16(b)) return KP_ERR_ARG;
  HIPCHK(launch_features(plan->P, b, features_out, reinterpret_cast<hipStream_t>(stream)));
  HIPCHK(hipEventRecord(plan->P.ev_last, reinterpret_cast<hipStream_t>(stream)));
  return KP_OK;
}

int opt_lambda(kp_plan_t plan, const float* b, const float* x_true, const double* grid,
               int ngrid, double* lambda_out, double* scores_out, void* stream) {
  if (!plan || !b || !x_true || !lambda_out || !valid_grid(grid, ngrid)) return KP_ERR_ARG;
  if (!aligned16(b) || !aligned16(x_true)) return KP_ERR_ARG;
  double sc[64];
  const int rc = spectral_call(plan, b, grid, ngrid, 1.0, 0.0, 2, sc, stream, x_true);
  if (rc != KP_OK) return rc;
  int best = 0;
  for (int g = 1; g < ngrid; ++g)
    if (sc[g] < sc[best]) best = g;
  *lambda_out = grid[best];
  if (scores_out) std::memcpy(scores_out, sc, sizeof(double) * ngrid);
  return KP_OK;
}

size_t mlp_workspace_size(int max_batch) {
  if (max_batch < 1 || max_batch > kMaxBatch) return 0;
  return model_bytes(max_batch);
}

int mlp_create(int max_batch, void* workspace, size_t ws_bytes, void* stream, kp_mlp_t* mlp) {
  if (!mlp) return KP_ERR_ARG;
  *mlp = nullptr;
  if (max_batch < 1 || max_batch > kMaxBatch) return KP_ERR_ARG;
  const size_t need = model_bytes(max_batch);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  kp_mlp_s* h = new (std::nothrow) kp_mlp_s();
  if (!h) return KP_ERR_ARG;
  Mlp& M = h->M;
  char* base = nullptr;
  if (workspace) {
    if (ws_bytes < need || !aligned16(workspace)) {
      delete h;
      return KP_ERR_WORKSPACE;
    }
    base = reinterpret_cast<char*>(workspace);
  } else {
    if (hipMalloc(&base, need) != hipSuccess) {
      delete h;
      return KP_ERR_HIP;
    }
    M.owns = true;
  }
  M.base = base;
  M.bytes = need;
  M.max_batch = max_batch;
  const size_t used = mlp_layout(max_batch, base, &M);
  h->feat1 = reinterpret_cast<float*>(base + used);
  h->pred1 = reinterpret_cast<double*>(base + used + 512);
  int rc = KP_OK;
  if (hipHostMalloc(reinterpret_cast<void**>(&M.host_loss), sizeof(double)) != hipSuccess)
    rc = KP_ERR_HIP;
  // zero parameters and moments; normaliser mean 0, scale 1
  if (rc == KP_OK && hipMemsetAsync(base, 0, used, s) != hipSuccess) rc = KP_ERR_HIP;
  if (rc == KP_OK) {
    std::vector<float> ones(MLP_NF, 1.0f);
    if (hipMemcpyAsync(M.scale, ones.data(), sizeof(float) * MLP_NF, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = KP_ERR_HIP;
  }
  // set-up of lambda_predict_noalloc on this device: the static array's
  // device address (the runtime makes the array resident here, so that the
  // entry point itself has nothing left to set up)
  void* sp = nullptr;
  if (rc == KP_OK) rc = scratch_address(&sp);
  if (rc != KP_OK) {
    if (M.host_loss) hipHostFree(M.host_loss);
    if (M.owns) hipFree(base);
    delete h;
    return rc;
  }
  *mlp = h;
  return KP_OK;
}

int mlp_set_params(kp_mlp_t mlp, const float* params, void* stream) {
  if (!mlp || !params) return KP_ERR_ARG;
  for (size_t i = 0; i < MLP_NPARAM; ++i)
    if (!std::isfinite(params[i])) return KP_ERR_ARG;
  Mlp& M = mlp->M;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipMemcpyAsync(M.params, params, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(M.m, 0, MLP_NPARAM * sizeof(float), s));
  HIPCHK(hipMemsetAsync(M.v, 0, MLP_NPARAM * sizeof(float), s));
  HIPCHK(mlp_refresh_half(M, s));
  HIPCHK(hipStreamSynchronize(s));
  M.step = 0;
  return KP_OK;
}

int mlp_get_params(kp_mlp_t mlp, float* params, void* stream) {
  if (!mlp || !params) return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipMemcpyAsync(params, mlp->M.params, MLP_NPARAM * sizeof(float),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

int mlp_set_normalizer(kp_mlp_t mlp, const float* mean, const float* scale, void* stream) {
  if (!mlp || !mean || !scale) return KP_ERR_ARG;
  for (int f = 0; f < MLP_NF; ++f)
    if (!std::isfinite(mean[f]) || !std::isfinite(scale[f]) || !(scale[f] > 0.0f))
      return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipMemcpyAsync(mlp->M.mu, mean, MLP_NF * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(mlp->M.scale, scale, MLP_NF * sizeof(float), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

int mlp_get_normalizer(kp_mlp_t mlp, float* mean, float* scale, void* stream) {
  if (!mlp || !mean || !scale) return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(hipMemcpyAsync(mean, mlp->M.mu, MLP_NF * sizeof(float), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(scale, mlp->M.scale, MLP_NF * sizeof(float), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return KP_OK;
}

int mlp_fit_normalizer(kp_mlp_t mlp, const float* features, int nb, void* stream) {
  if (!mlp || !features || nb < 1) return KP_ERR_ARG;
  HIPCHK(mlp_fit_norm(mlp->M, features, nb, reinterpret_cast<hipStream_t>(stream)));
  return KP_OK;
}

int lambda_predict(kp_mlp_t mlp, const float* features, int nb, double* log10_lambda,
                   void* stream) {
  if (!mlp || !features || !log10_lambda || nb < 1) return KP_ERR_ARG;
  if (!aligned16(features)) return KP_ERR_ARG;
  const Mlp& M = mlp->M;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int off = 0; off < nb; off += M.max_batch) {
    const int cnt = nb - off < M.max_batch ? nb - off : M.max_batch;
    HIPCHK(mlp_forward(M, features + (size_t)off * MLP_NF, nullptr, cnt, log10_lambda + off, s));
  }
  return KP_OK;
}

int lambda_predict_noalloc(kp_mlp_t mlp, const float* features, int nb, double* log10_lambda,
                           void* stream) {
  if (!mlp || !features || !log10_lambda || nb < 1) return KP_ERR_ARG;
  if (!aligned16(features)) return KP_ERR_ARG;
  if (nb > KP_PREDICT_NOALLOC_MAX_ROWS) return KP_ERR_WORKSPACE;
  void* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc != KP_OK) return rc;
  // the model's weights and normaliser; activations in the static array
  Mlp Q = mlp->M;
  Q.max_batch = KP_PREDICT_NOALLOC_MAX_ROWS;
  if (mlp_act_layout(KP_PREDICT_NOALLOC_MAX_ROWS, reinterpret_cast<char*>(base), &Q) >
      kNoallocBytes)
    return KP_ERR_WORKSPACE;
  HIPCHK(mlp_forward(Q, features, nullptr, nb, log10_lambda,
                     reinterpret_cast<hipStream_t>(stream)));
  return KP_OK;
}

int mlp_train_step(kp_mlp_t mlp, const float* features, const float* targets, int nrows,
                   const int* rows, int nb, float lr, double* loss_out, void* stream) {
  if (!mlp || !features || !targets || nrows < 1 || nb < 1) return KP_ERR_ARG;
  Mlp& M = mlp->M;
  if (nb > M.max_batch || !(lr > 0.0f) || !std::isfinite(lr)) return KP_ERR_ARG;
  if (!aligned16(features)) return KP_ERR_ARG;
  if (rows) {
    for (int i = 0; i < nb; ++i)
      if (rows[i] < 0 || rows[i] >= nrows) return KP_ERR_ARG;
  } else if (nb > nrows) {
    return KP_ERR_ARG;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int* rows_dev = nullptr;
  if (rows) {
    HIPCHK(hipMemcpyAsync(M.rows, rows, sizeof(int) * nb, hipMemcpyHostToDevice, s));
    rows_dev = M.rows;
  }
  HIPCHK(mlp_forward(M, features, rows_dev, nb, nullptr, s));
  HIPCHK(mlp_backward(M, targets, rows_dev, nb, s));
  M.step += 1;
  const float bc1 = (float)(1.0 - std::pow((double)kBeta1, (double)M.step));
  const float bc2 = (float)(1.0 - std::pow((double)kBeta2, (double)M.step));
  HIPCHK(mlp_adam(M, lr, kBeta1, kBeta2, kEps, bc1, bc2, s));
  if (loss_out) return read_loss(M, loss_out, s);
  return KP_OK;
}

int mlp_gradients(kp_mlp_t mlp, const float* features, const float* targets, int nb,
                  float* grads, double* loss_out, void* stream) {
  if (!mlp || !features || !targets || !grads || nb < 1) return KP_ERR_ARG;
  const Mlp& M = mlp->M;
  if (nb > M.max_batch || !aligned16(features)) return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHK(mlp_forward(M, features, nullptr, nb, nullptr, s));
  HIPCHK(mlp_backward(M, targets, nullptr, nb, s));
  HIPCHK(hipMemcpyAsync(grads, M.grads, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
  double loss = 0.0;
  const int rc = read_loss(M, &loss, s);
  if (rc != KP_OK) return rc;
  if (loss_out) *loss_out = loss;
  return KP_OK;
}

int mlp_destroy(kp_mlp_t mlp) {
  if (!mlp) return KP_ERR_ARG;
  Mlp& M = mlp->M;
  if (M.host_loss) hipHostFree(M.host_loss);
  if (M.owns) hipFree(M.base);
  delete mlp;
  return KP_OK;
}

int kp_lambda_learned(kp_plan_t plan, kp_mlp_t mlp, const float* b, const double* grid,
                      int ngrid, double tau, kp_lambda_info_t* info, void* stream) {
  if (!plan || !mlp || !b || !info || !valid_grid(grid, ngrid, 63)) return KP_ERR_ARG;
  if (!(tau >= 0.0) || !std::isfinite(tau) || !aligned16(b)) return KP_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Mlp& M = mlp->M;
  HIPCHK(launch_features(plan->P, b, mlp->feat1, s));
  HIPCHK(mlp_forward(M, mlp->feat1, nullptr, 1, mlp->pred1, s));
  double y = 0.0;
  HIPCHK(hipMemcpyAsync(M.host_loss, mlp->pred1, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  y = *M.host_loss;
  if (!std::isfinite(y)) return KP_ERR_SOLVER;
  double lo = grid[0], hi = grid[0];
  for (int g = 1; g < ngrid; ++g) {
    lo = grid[g] < lo ? grid[g] : lo;
    hi = grid[g] > hi ? grid[g] : hi;
  }
  double lp = std::pow(10.0, y);
  lp = lp < lo ? lo : (lp > hi ? hi : lp);
  double g2[64], sc[64];
  std::memcpy(g2, grid, sizeof(double) * ngrid);
  g2[ngrid] = lp;
  const int rc = spectral_call(plan, b, g2, ngrid + 1, 1.0, 0.0, 0, sc, stream);
  if (rc != KP_OK) return rc;
  int best = 0;
  for (int g = 1; g < ngrid; ++g)
    if (sc[g] < sc[best]) best = g;
  // zero data: every score is 0 and the prediction is as good as any
  const double ratio = sc[best] > 0.0 ? sc[ngrid] / sc[best] - 1.0
                                      : (sc[ngrid] > 0.0 ? HUGE_VAL : 0.0);
  info->lambda_pred = lp;
  info->lambda_gcv = grid[best];
  info->gcv_ratio = ratio;
  info->fell_back = ratio > tau ? 1 : 0;
  info->lambda = info->fell_back ? grid[best] : lp;
  info->reserved = 0;
  return KP_OK;
}

}  // extern "C"
