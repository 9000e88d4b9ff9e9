// Host side of the learned-guess network (C ABI in include/ddps.h).
//
// Four layers d_in -> H -> H -> H -> d_out with ReLU between them.
// Parameters are one packed FP32 vector [W1, b1, W2, b2, W3, b3, W4, b4]
// (W_l row-major, fan-in x fan-out); a bf16 copy of it feeds the products.
// Activations are stored in bf16, every product accumulates in FP32, and
// training minimises the mean squared error with Adam on the FP32 master
// parameters.
#include "../../include/ddps.h"
#include "ddps_mlp_internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using namespace ddps;

struct ddps_mlp_ctx {
  int d_in = 0, H = 0, d_out = 0, max_batch = 0;
  hipStream_t stream = nullptr;
  int64_t off[8] = {}, count = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  __bf16* pb = nullptr;
  __bf16 *X0 = nullptr, *A1 = nullptr, *A2 = nullptr, *A3 = nullptr, *dYb = nullptr, *dZ = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *Y = nullptr, *dA = nullptr;
  double* part = nullptr;
  double* h_part = nullptr;
  int adam_t = 0;
  std::vector<void*> allocs;
  template <typename T>
  bool alloc(T*& ptr, int64_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess) return false;
    allocs.push_back(q);
    ptr = (T*)q;
    return true;
  }
  const __bf16* W(int l) const { return pb + off[2 * l]; }
  const float* b(int l) const { return p + off[2 * l + 1]; }
  int fan_in(int l) const { return l == 0 ? d_in : H; }
  int fan_out(int l) const { return l == 3 ? d_out : H; }
};

namespace {

// splitmix64 (Steele, Lea & Flood 2014): initial weights only
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int forward(ddps_mlp_ctx* M, int B, const float* X) {
  hipStream_t s = M->stream;
  mlp_to_bf16((int64_t)B * M->d_in, X, M->X0, s);
  mlp_gemm(false, false, B, M->H, M->d_in, M->X0, M->d_in, M->W(0), M->H, M->b(0), MLP_BIAS | MLP_F32 | MLP_RELU_BF16,
           M->Z1, M->A1, M->H, s);
  mlp_gemm(false, false, B, M->H, M->H, M->A1, M->H, M->W(1), M->H, M->b(1), MLP_BIAS | MLP_F32 | MLP_RELU_BF16,
           M->Z2, M->A2, M->H, s);
  mlp_gemm(false, false, B, M->H, M->H, M->A2, M->H, M->W(2), M->H, M->b(2), MLP_BIAS | MLP_F32 | MLP_RELU_BF16,
           M->Z3, M->A3, M->H, s);
  mlp_gemm(false, false, B, M->d_out, M->H, M->A3, M->H, M->W(3), M->d_out, M->b(3), MLP_BIAS | MLP_F32, M->Y,
           nullptr, M->d_out, s);
  return hipGetLastError() == hipSuccess ? DDPS_OK : DDPS_E_HIP;
}

// gradients of mean((Y - T)^2) into M->g; returns the loss through *loss
int backward(ddps_mlp_ctx* M, int B, const float* T, double* loss) {
  hipStream_t s = M->stream;
  const int64_t ny = (int64_t)B * M->d_out;
  const int W = mlp_mse(ny, 1.f / (float)ny, M->Y, T, M->dYb, M->part, s);
  float* g = M->g;
  const __bf16* acts[4] = {M->X0, M->A1, M->A2, M->A3};
  const float* Zs[3] = {M->Z1, M->Z2, M->Z3};
  const __bf16* dcur = M->dYb;   // dZ of layer l (bf16), batch x fan_out(l)
  for (int l = 3; l >= 0; --l) {
    const int fi = M->fan_in(l), fo = M->fan_out(l);
    // dW_l = act_{l}^T dZ_l   (fan_in x fan_out)
    mlp_gemm(true, false, fi, fo, B, acts[l], fi, dcur, fo, nullptr, MLP_F32, g + M->off[2 * l], nullptr, fo, s);
    mlp_bias_grad(B, fo, dcur, g + M->off[2 * l + 1], s);
    if (l == 0) break;
    // dA_{l-1} = dZ_l W_l^T  (batch x fan_in), then dZ_{l-1} = dA * (Z_{l-1} > 0)
    mlp_gemm(false, true, B, fi, fo, dcur, fo, M->W(l), fo, nullptr, MLP_F32, M->dA, nullptr, fi, s);
    __bf16* dz = (l % 2 == 1) ? M->dZ : M->dZ + (int64_t)M->max_batch * M->H;
    mlp_relu_bwd((int64_t)B * fi, M->dA, Zs[l - 1], dz, s);
    dcur = dz;
  }
  if (hipGetLastError() != hipSuccess) return DDPS_E_HIP;
  if (loss) {
    if (hipMemcpyAsync(M->h_part, M->part, sizeof(double) * W, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return DDPS_E_HIP;
    double acc = 0;
    for (int i = 0; i < W; ++i) acc += M->h_part[i];
    *loss = acc / (double)ny;
  }
  return DDPS_OK;
}

}  // namespace

namespace ddps {
int mlp_shape(const ddps_mlp_ctx* M, int* d_in, int* d_out, int* max_batch, hipStream_t* stream) {
  if (!M) return DDPS_E_ARG;
  *d_in = M->d_in;
  *d_out = M->d_out;
  *max_batch = M->max_batch;
  *stream = M->stream;
  return DDPS_OK;
}
}  // namespace ddps

extern "C" {

int ddps_mlp_create(ddps_mlp* out, int32_t d_in, int32_t hidden, int32_t d_out, int32_t max_batch, uint64_t seed,
                    void* stream) {
  if (!out || d_in < 1 || hidden < 1 || d_out < 1 || max_batch < 1) return DDPS_E_ARG;
  *out = nullptr;
  ddps_mlp_ctx* M = new (std::nothrow) ddps_mlp_ctx();
  if (!M) return DDPS_E_NOMEM;
  M->d_in = d_in;
  M->H = hidden;
  M->d_out = d_out;
  M->max_batch = max_batch;
  M->stream = (hipStream_t)stream;
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    M->off[2 * l] = o;
    o += (int64_t)M->fan_in(l) * M->fan_out(l);
    M->off[2 * l + 1] = o;
    o += M->fan_out(l);
  }
  M->count = o;
  const int64_t B = max_batch, wide = std::max<int64_t>(std::max(hidden, d_in), d_out);
  bool ok = M->alloc(M->p, o) && M->alloc(M->g, o) && M->alloc(M->m, o) && M->alloc(M->v, o) && M->alloc(M->pb, o) &&
            M->alloc(M->X0, B * d_in) && M->alloc(M->A1, B * hidden) && M->alloc(M->A2, B * hidden) &&
            M->alloc(M->A3, B * hidden) && M->alloc(M->dYb, B * d_out) && M->alloc(M->dZ, 2 * B * hidden) &&
            M->alloc(M->Z1, B * hidden) && M->alloc(M->Z2, B * hidden) && M->alloc(M->Z3, B * hidden) &&
            M->alloc(M->Y, B * d_out) && M->alloc(M->dA, B * wide) && M->alloc(M->part, 256);
  if (!ok || hipHostMalloc((void**)&M->h_part, 256 * sizeof(double)) != hipSuccess) {
    ddps_mlp_destroy(M);
    return DDPS_E_NOMEM;
  }
  // He-uniform weights from the seed, zero biases
  std::vector<float> h(o, 0.f);
  uint64_t st = seed;
  for (int l = 0; l < 4; ++l) {
    const double lim = std::sqrt(6.0 / M->fan_in(l));
    for (int64_t q = M->off[2 * l]; q < M->off[2 * l + 1]; ++q) {
      const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
      h[q] = (float)((2.0 * u - 1.0) * lim);
    }
  }
  *out = M;
  return ddps_mlp_set_params(M, h.data());
}

int64_t ddps_mlp_param_count(ddps_mlp M) { return M ? M->count : -1; }

int ddps_mlp_set_params(ddps_mlp M, const float* host_params) {
  if (!M || !host_params) return DDPS_E_ARG;
  hipStream_t s = M->stream;
  if (hipMemcpyAsync(M->p, host_params, sizeof(float) * M->count, hipMemcpyHostToDevice, s) != hipSuccess)
    return DDPS_E_HIP;
  mlp_to_bf16(M->count, M->p, M->pb, s);
  // fresh optimiser state
  std::vector<float> z(M->count, 0.f);
  if (hipMemcpyAsync(M->m, z.data(), sizeof(float) * M->count, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(M->v, z.data(), sizeof(float) * M->count, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DDPS_E_HIP;
  M->adam_t = 0;
  return DDPS_OK;
}

int ddps_mlp_get_params(ddps_mlp M, float* host_params) {
  if (!M || !host_params) return DDPS_E_ARG;
  if (hipMemcpyAsync(host_params, M->p, sizeof(float) * M->count, hipMemcpyDeviceToHost, M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return DDPS_E_HIP;
  return DDPS_OK;
}

int ddps_mlp_forward(ddps_mlp M, int32_t batch, const float* X, float* Y) {
  if (!M || !X || !Y || batch < 1 || batch > M->max_batch) return DDPS_E_ARG;
  int rc = forward(M, batch, X);
  if (rc) return rc;
  if (hipMemcpyAsync(Y, M->Y, sizeof(float) * batch * M->d_out, hipMemcpyDeviceToDevice, M->stream) != hipSuccess)
    return DDPS_E_HIP;
  return DDPS_OK;
}

int ddps_mlp_gradients(ddps_mlp M, int32_t batch, const float* X, const float* T, float* host_grads, double* loss) {
  if (!M || !X || !T || batch < 1 || batch > M->max_batch) return DDPS_E_ARG;
  int rc = forward(M, batch, X);
  if (rc) return rc;
  if ((rc = backward(M, batch, T, loss))) return rc;
  if (host_grads) {
    if (hipMemcpyAsync(host_grads, M->g, sizeof(float) * M->count, hipMemcpyDeviceToHost, M->stream) != hipSuccess ||
        hipStreamSynchronize(M->stream) != hipSuccess)
      return DDPS_E_HIP;
  }
  return DDPS_OK;
}

int ddps_mlp_train_step(ddps_mlp M, int32_t batch, const float* X, const float* T, float lr, double* loss) {
  if (!M || !X || !T || batch < 1 || batch > M->max_batch || !(lr > 0.f)) return DDPS_E_ARG;
  int rc = forward(M, batch, X);
  if (rc) return rc;
  if ((rc = backward(M, batch, T, loss))) return rc;
  M->adam_t += 1;
  mlp_adam(M->count, lr, 0.9f, 0.999f, 1e-8f, M->adam_t, M->p, M->g, M->m, M->v, M->pb, M->stream);
  return hipGetLastError() == hipSuccess ? DDPS_OK : DDPS_E_HIP;
}

void ddps_mlp_destroy(ddps_mlp M) {
  if (!M) return;
  if (M->stream) (void)hipStreamSynchronize(M->stream);
  for (void* q : M->allocs) (void)hipFree(q);
  if (M->h_part) (void)hipHostFree(M->h_part);
  delete M;
}

}  // extern "C"
