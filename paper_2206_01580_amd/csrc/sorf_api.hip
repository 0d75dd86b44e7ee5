// C ABI entry points: host-side argument validation, then kernel launches on
// the caller's stream. Nothing here allocates device memory or synchronises.
#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/sorf.h"
#include "sorf_internal.h"

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// float4 loads and stores need 16-byte aligned rows
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

constexpr int32_t kMaxSolveD = 32768;

sorf_status check_model(const sorf_model* m) {
  if (m == nullptr) return SORF_ERR_INVALID_ARG;
  if (m->d < 2 || m->d > 1024 || !is_pow2(m->d)) return SORF_ERR_INVALID_ARG;
  if (m->n_stacks < 1 || m->n_elements < 1) return SORF_ERR_INVALID_ARG;
  if (m->n_transforms < 1 || m->n_transforms > 3) return SORF_ERR_INVALID_ARG;
  if (!(m->sigma > 0.0f) || !std::isfinite(m->sigma)) return SORF_ERR_INVALID_ARG;
  if (int64_t(m->d) * m->n_stacks > (int64_t(1) << 20)) return SORF_ERR_INVALID_ARG;
  if (m->signs == nullptr || m->bias == nullptr) return SORF_ERR_INVALID_ARG;
  if (!aligned16(m->bias) || (reinterpret_cast<uintptr_t>(m->signs) & 3u)) return SORF_ERR_INVALID_ARG;
  return SORF_OK;
}

sorf_status check_batch(const sorf_batch* b) {
  if (b == nullptr) return SORF_ERR_INVALID_ARG;
  if (b->n_atoms < 0 || b->n_mols < 0) return SORF_ERR_INVALID_ARG;
  if (b->n_atoms > (int64_t(1) << 40) || b->n_mols > (int64_t(1) << 31) - 1) return SORF_ERR_INVALID_ARG;
  if (b->mol_ptr == nullptr) return SORF_ERR_INVALID_ARG;
  if (b->n_atoms > 0 && (b->x == nullptr || b->element == nullptr)) return SORF_ERR_INVALID_ARG;
  if (!aligned16(b->x)) return SORF_ERR_INVALID_ARG;
  return SORF_OK;
}

SorfFeatureArgs pack(const sorf_model* m, const sorf_batch* b) {
  SorfFeatureArgs a;
  a.d = m->d;
  a.n_stacks = m->n_stacks;
  a.n_transforms = m->n_transforms;
  a.n_elements = m->n_elements;
  a.sigma = m->sigma;
  a.signs = m->signs;
  a.bias = m->bias;
  a.x = b->x;
  a.element = b->element;
  a.mol_ptr = b->mol_ptr;
  a.n_atoms = b->n_atoms;
  a.n_mols = b->n_mols;
  return a;
}

sorf_status dev(hipError_t e) { return e == hipSuccess ? SORF_OK : SORF_ERR_DEVICE; }

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// chunk offsets [n_mols + 1] and chunk partials [chunks][n_stacks] of the
// energies-only path
size_t energy_ws(const sorf_model* m, int64_t n_atoms, int64_t n_mols) {
  return align256(sizeof(int64_t) * size_t(n_mols + 1)) +
         align256(sizeof(float) * size_t(energy_chunk_bound(n_atoms, n_mols)) *
                  size_t(m->n_stacks));
}

// [e_atom | grad | force plan] for energies with forces; the energies-only
// path uses the energy_ws() bytes at the end.
size_t predict_ws(const sorf_model* m, int64_t n_atoms, int64_t n_mols) {
  return align256(sizeof(float) * size_t(n_atoms)) +
         align256(sizeof(float) * size_t(n_atoms) * size_t(m->d)) +
         sorf_force_plan_bytes(n_atoms, n_mols) + energy_ws(m, n_atoms, n_mols);
}

}  // namespace

extern "C" {

int32_t sorf_abi_version(void) { return SORF_ABI_VERSION; }

const char* sorf_status_string(sorf_status s) {
  switch (s) {
    case SORF_OK: return "SORF_OK";
    case SORF_ERR_INVALID_ARG: return "SORF_ERR_INVALID_ARG";
    case SORF_ERR_UNSUPPORTED: return "SORF_ERR_UNSUPPORTED";
    case SORF_ERR_DEVICE: return "SORF_ERR_DEVICE";
    case SORF_ERR_WORKSPACE: return "SORF_ERR_WORKSPACE";
    case SORF_ERR_BUSY: return "SORF_ERR_BUSY";
  }
  return "SORF_ERR_UNKNOWN";
}

sorf_status sorf_forward(const sorf_model* model, const sorf_batch* batch, float* Z,
                         sorf_stream_t stream) {
  sorf_status s = check_model(model);
  if (s != SORF_OK) return s;
  if ((s = check_batch(batch)) != SORF_OK) return s;
  if (batch->n_mols > 0 && Z == nullptr) return SORF_ERR_INVALID_ARG;
  if (!aligned16(Z)) return SORF_ERR_INVALID_ARG;
  return dev(sorf_launch_forward(pack(model, batch), Z, hipStream_t(stream)));
}

sorf_status sorf_backward(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                          const float* dE, float* grad_x, sorf_stream_t stream) {
  sorf_status s = check_model(model);
  if (s != SORF_OK) return s;
  if ((s = check_batch(batch)) != SORF_OK) return s;
  if (batch->n_atoms > 0 && (alpha == nullptr || grad_x == nullptr)) return SORF_ERR_INVALID_ARG;
  if (!aligned16(alpha) || !aligned16(grad_x)) return SORF_ERR_INVALID_ARG;
  return dev(sorf_launch_atom_adjoint(pack(model, batch), alpha, dE, grad_x, nullptr,
                                      hipStream_t(stream)));
}

size_t sorf_energy_grad_workspace_bytes(int64_t n_atoms) {
  if (n_atoms < 0 || n_atoms > (int64_t(1) << 40)) return 0;
  return ((sizeof(float) * size_t(n_atoms)) + 255) & ~size_t(255);
}

sorf_status sorf_energy_grad(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                             float* E, float* grad_x, void* workspace, size_t workspace_bytes,
                             sorf_stream_t stream) {
  sorf_status s = check_model(model);
  if (s != SORF_OK) return s;
  if ((s = check_batch(batch)) != SORF_OK) return s;
  if (batch->n_mols > 0 && E == nullptr) return SORF_ERR_INVALID_ARG;
  if (batch->n_atoms > 0 && (alpha == nullptr || grad_x == nullptr)) return SORF_ERR_INVALID_ARG;
  if (!aligned16(alpha) || !aligned16(grad_x)) return SORF_ERR_INVALID_ARG;
  const size_t need = sorf_energy_grad_workspace_bytes(batch->n_atoms);
  if (batch->n_atoms > 0 && (workspace == nullptr || workspace_bytes < need))
    return SORF_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  return dev(sorf_launch_energy_grad(pack(model, batch), alpha, grad_x,
                                     static_cast<float*>(workspace), E, hipStream_t(stream)));
}

sorf_status sorf_derivative_features(const sorf_model* model, const sorf_batch* batch,
                                     const float* J, const int64_t* J_ptr, float* dZ,
                                     sorf_stream_t stream) {
  sorf_status s = check_model(model);
  if (s != SORF_OK) return s;
  if ((s = check_batch(batch)) != SORF_OK) return s;
  if (batch->n_atoms > 0 && (J == nullptr || J_ptr == nullptr || dZ == nullptr))
    return SORF_ERR_INVALID_ARG;
  if (!aligned16(dZ)) return SORF_ERR_INVALID_ARG;
  return dev(sorf_launch_dz(pack(model, batch), J, J_ptr, dZ, hipStream_t(stream)));
}

size_t sorf_project_workspace_bytes(int64_t n_atoms, int32_t n_elements) {
  if (n_atoms < 0 || n_atoms > (int64_t(1) << 40) || n_elements < 1 || n_elements > 256) return 0;
  return sorf_project_ws_bytes(n_atoms, n_elements);
}

sorf_status sorf_project(int64_t n_atoms, int32_t d_rep, const float* rho, const int32_t* element,
                         int32_t n_elements, const float* U, int32_t d, float* x,
                         void* workspace, size_t workspace_bytes, sorf_stream_t stream) {
  if (n_atoms < 0 || n_atoms > (int64_t(1) << 40)) return SORF_ERR_INVALID_ARG;
  if (d_rep < 1 || d < 1 || d > (1 << 20) || n_elements < 1) return SORF_ERR_INVALID_ARG;
  if (n_elements > 256) return SORF_ERR_UNSUPPORTED;
  if (int64_t(d_rep) * d * n_elements > (int64_t(1) << 40)) return SORF_ERR_INVALID_ARG;
  if (n_atoms == 0) return SORF_OK;
  if (rho == nullptr || element == nullptr || U == nullptr || x == nullptr)
    return SORF_ERR_INVALID_ARG;
  const size_t need = sorf_project_ws_bytes(n_atoms, n_elements);
  if (workspace == nullptr || workspace_bytes < need) return SORF_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  return dev(sorf_launch_project(n_atoms, d_rep, rho, element, n_elements, U, d, x, workspace,
                                 hipStream_t(stream)));
}

size_t sorf_projection_fit_workspace_bytes(int32_t d_rep) {
  if (d_rep < 1 || d_rep > 4096) return 0;
  return sorf_fit_ws_bytes(d_rep);
}

sorf_status sorf_projection_fit(int64_t n_samples, int32_t d_rep, const float* sample,
                                int32_t n_pca, float* U, double* singular_values,
                                void* workspace, size_t workspace_bytes, sorf_stream_t stream) {
  if (d_rep < 1 || n_pca < 1 || n_pca > d_rep || n_samples < 0) return SORF_ERR_INVALID_ARG;
  if (d_rep > 4096) return SORF_ERR_UNSUPPORTED;
  if (n_samples > (int64_t(1) << 40)) return SORF_ERR_INVALID_ARG;
  if (U == nullptr || (n_samples > 0 && sample == nullptr)) return SORF_ERR_INVALID_ARG;
  const size_t need = sorf_fit_ws_bytes(d_rep);
  if (workspace == nullptr || workspace_bytes < need) return SORF_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  return dev(sorf_launch_projection_fit(n_samples, d_rep, sample, n_pca, U, singular_values,
                                        workspace, hipStream_t(stream)));
}

static bool fchl_params_ok(const sorf_fchl19_params* p) {
  if (p == nullptr || p->n2 < 1 || p->n3 < 2 || p->n2 > 4096 || p->n3 > 4096) return false;
  const float v[] = {p->eta2, p->eta3, p->N2, p->N3, p->c3, p->zeta, p->rcut};
  for (float x : v)
    if (!std::isfinite(x)) return false;
  return p->eta2 > 0.0f && p->eta3 > 0.0f && p->rcut > 0.0f;
}

int64_t sorf_fchl19_length(int32_t n_elements, const sorf_fchl19_params* params) {
  if (n_elements < 1 || n_elements > 16 || !fchl_params_ok(params)) return 0;
  return sorf_fchl19_len(n_elements, params->n2, params->n3);
}

sorf_status sorf_fchl19_forward(const float* R, const int32_t* element, const int64_t* mol_ptr,
                                int64_t n_atoms, int64_t n_mols, int32_t n_elements,
                                const sorf_fchl19_params* params, float* rho,
                                sorf_stream_t stream) {
  if (n_atoms < 0 || n_mols < 0 || n_atoms > (int64_t(1) << 40)) return SORF_ERR_INVALID_ARG;
  if (n_elements < 1 || !fchl_params_ok(params)) return SORF_ERR_INVALID_ARG;
  if (n_elements > 16) return SORF_ERR_UNSUPPORTED;
  if (n_atoms == 0) return SORF_OK;
  if (R == nullptr || element == nullptr || mol_ptr == nullptr || rho == nullptr || n_mols == 0)
    return SORF_ERR_INVALID_ARG;
  const FchlParamsHost p{params->n2, params->n3, params->eta2, params->eta3, params->N2,
                         params->N3, params->c3, params->zeta, params->rcut};
  return dev(sorf_launch_fchl19_forward(R, element, mol_ptr, n_atoms, n_mols, n_elements, p, rho,
                                        hipStream_t(stream)));
}

sorf_status sorf_fchl19_backward(const float* R, const int32_t* element, const int64_t* mol_ptr,
                                 int64_t n_atoms, int64_t n_mols, int32_t n_elements,
                                 const sorf_fchl19_params* params, const float* g, float* dR,
                                 sorf_stream_t stream) {
  if (n_atoms < 0 || n_mols < 0 || n_atoms > (int64_t(1) << 40)) return SORF_ERR_INVALID_ARG;
  if (n_mols > (int64_t(1) << 31) - 1) return SORF_ERR_INVALID_ARG;
  if (n_elements < 1 || !fchl_params_ok(params)) return SORF_ERR_INVALID_ARG;
  if (n_elements > 16) return SORF_ERR_UNSUPPORTED;
  if (n_atoms == 0) return SORF_OK;
  if (R == nullptr || element == nullptr || mol_ptr == nullptr || g == nullptr || dR == nullptr ||
      n_mols == 0)
    return SORF_ERR_INVALID_ARG;
  const FchlParamsHost p{params->n2, params->n3, params->eta2, params->eta3, params->N2,
                         params->N3, params->c3, params->zeta, params->rcut};
  return dev(sorf_launch_fchl19_backward(R, element, mol_ptr, n_mols, n_elements, p, g, dR,
                                         hipStream_t(stream)));
}

size_t sorf_gram_workspace_bytes(int64_t n_rows, int32_t D, sorf_gram_precision precision) {
  if (n_rows < 0 || D < 1 || D > (1 << 20)) return 0;
  if (int(precision) < 0 || int(precision) > 5) return 0;
  return sorf_gram_ws_bytes(n_rows, D, int(precision));
}

sorf_status sorf_gram_accumulate(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                 sorf_gram_precision precision, int32_t scale_exp, float* G,
                                 float* Zty, void* workspace, size_t workspace_bytes,
                                 sorf_stream_t stream) {
  if (n_rows < 0 || D < 1 || D > (1 << 20)) return SORF_ERR_INVALID_ARG;
  if (int(precision) < 0 || int(precision) > 5) return SORF_ERR_INVALID_ARG;
  if (scale_exp < -60 || scale_exp > 60) return SORF_ERR_INVALID_ARG;
  if (scale_exp != 0 && precision != SORF_GRAM_FP16 && precision != SORF_GRAM_FP16_HILO)
    return SORF_ERR_INVALID_ARG;
  if (G == nullptr) return SORF_ERR_INVALID_ARG;
  if (n_rows > 0 && Z == nullptr) return SORF_ERR_INVALID_ARG;
  if (y != nullptr && Zty == nullptr) return SORF_ERR_INVALID_ARG;
  if (!aligned16(Z)) return SORF_ERR_INVALID_ARG;
  if (int64_t(D) * D > (int64_t(1) << 36)) return SORF_ERR_UNSUPPORTED;
  hipStream_t st = hipStream_t(stream);
  if (n_rows == 0) return SORF_OK;
  const size_t need = sorf_gram_ws_bytes(n_rows, D, int(precision));
  if (need > 0) {
    if (workspace == nullptr || workspace_bytes < need) return SORF_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  }
  return dev(sorf_launch_gram(n_rows, D, Z, y, int(precision), scale_exp, G, Zty, workspace, st));
}

sorf_status sorf_gram_accumulate_f64(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                     double* G, double* Zty, sorf_stream_t stream) {
  if (n_rows < 0 || D < 1 || D > (1 << 20)) return SORF_ERR_INVALID_ARG;
  if (G == nullptr) return SORF_ERR_INVALID_ARG;
  if (n_rows > 0 && Z == nullptr) return SORF_ERR_INVALID_ARG;
  if (y != nullptr && Zty == nullptr) return SORF_ERR_INVALID_ARG;
  if (!aligned16(Z)) return SORF_ERR_INVALID_ARG;
  if (int64_t(D) * D > (int64_t(1) << 35)) return SORF_ERR_UNSUPPORTED;
  hipStream_t st = hipStream_t(stream);
  if (n_rows == 0) return SORF_OK;
  return dev(sorf_launch_gram_f64(n_rows, D, Z, y, G, Zty, st));
}

size_t sorf_gram_split_workspace_bytes(int64_t n_rows, int32_t D) {
  if (n_rows < 0 || D < 1 || D > (1 << 20)) return 0;
  return sorf_gram_split_ws_bytes(n_rows, D);
}

sorf_status sorf_gram_accumulate_split(int64_t n_rows, int32_t D, const float* Z, const float* y,
                                       double* G, double* Zty, void* workspace,
                                       size_t workspace_bytes, sorf_stream_t stream) {
  if (n_rows < 0 || D < 1 || D > (1 << 20)) return SORF_ERR_INVALID_ARG;
  if (G == nullptr) return SORF_ERR_INVALID_ARG;
  if (n_rows > 0 && Z == nullptr) return SORF_ERR_INVALID_ARG;
  if (y != nullptr && Zty == nullptr) return SORF_ERR_INVALID_ARG;
  if (!aligned16(Z)) return SORF_ERR_INVALID_ARG;
  if (int64_t(D) * D > (int64_t(1) << 35)) return SORF_ERR_UNSUPPORTED;
  if (n_rows == 0) return SORF_OK;
  const size_t need = sorf_gram_split_ws_bytes(n_rows, D);
  if (workspace == nullptr || workspace_bytes < need) return SORF_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  return dev(sorf_launch_gram_split(n_rows, D, Z, y, G, Zty, workspace, hipStream_t(stream)));
}

size_t sorf_solve_workspace_bytes(int32_t D) {
  if (D < 1 || D > kMaxSolveD) return 0;
  return sorf_solve_ws_bytes(D);
}

namespace {

sorf_status check_solve(int32_t D, const void* G, const void* Zty, double lambda,
                        int32_t n_refine, const double* alpha, const int32_t* info,
                        const void* workspace, size_t workspace_bytes) {
  if (D < 1 || D > kMaxSolveD) return SORF_ERR_INVALID_ARG;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return SORF_ERR_INVALID_ARG;
  if (n_refine < 0 || n_refine > 16) return SORF_ERR_INVALID_ARG;
  if (G == nullptr || Zty == nullptr || alpha == nullptr || info == nullptr)
    return SORF_ERR_INVALID_ARG;
  if (workspace == nullptr || workspace_bytes < sorf_solve_ws_bytes(D)) return SORF_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  return SORF_OK;
}

// the side stream must differ from the call's stream and come with both events
sorf_status check_streams(const sorf_solve_streams* s, sorf_stream_t stream) {
  if (s == nullptr) return SORF_OK;
  if (s->side == nullptr || s->event_fork == nullptr || s->event_join == nullptr)
    return SORF_ERR_INVALID_ARG;
  if (s->side == stream || s->event_fork == s->event_join) return SORF_ERR_INVALID_ARG;
  return SORF_OK;
}

}  // namespace

sorf_status sorf_solve_streams_create(sorf_solve_streams* s) {
  if (s == nullptr) return SORF_ERR_INVALID_ARG;
  s->side = nullptr;
  s->event_fork = s->event_join = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return SORF_ERR_DEVICE;
  if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(st);
    return SORF_ERR_DEVICE;
  }
  if (hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(a);
    (void)hipStreamDestroy(st);
    return SORF_ERR_DEVICE;
  }
  s->side = st;
  s->event_fork = a;
  s->event_join = b;
  return SORF_OK;
}

sorf_status sorf_solve_streams_destroy(sorf_solve_streams* s) {
  if (s == nullptr) return SORF_ERR_INVALID_ARG;
  hipError_t e = hipSuccess, t;
  if (s->side != nullptr && (t = hipStreamSynchronize(hipStream_t(s->side))) != hipSuccess) e = t;
  if (s->event_fork != nullptr && (t = hipEventDestroy(hipEvent_t(s->event_fork))) != hipSuccess) e = t;
  if (s->event_join != nullptr && (t = hipEventDestroy(hipEvent_t(s->event_join))) != hipSuccess) e = t;
  if (s->side != nullptr && (t = hipStreamDestroy(hipStream_t(s->side))) != hipSuccess) e = t;
  s->side = nullptr;
  s->event_fork = s->event_join = nullptr;
  return dev(e);
}

sorf_status sorf_solve_streamed(int32_t D, const float* G, const float* Zty, double lambda,
                                int32_t n_refine, double* alpha, int32_t* info, void* workspace,
                                size_t workspace_bytes, const sorf_solve_streams* streams,
                                sorf_stream_t stream) {
  sorf_status s = check_solve(D, G, Zty, lambda, n_refine, alpha, info, workspace,
                              workspace_bytes);
  if (s != SORF_OK) return s;
  if ((s = check_streams(streams, stream)) != SORF_OK) return s;
  return dev(sorf_launch_solve(D, G, Zty, lambda, n_refine, alpha, info, workspace,
                               hipStream_t(stream),
                               streams ? hipStream_t(streams->side) : nullptr,
                               streams ? hipEvent_t(streams->event_fork) : nullptr,
                               streams ? hipEvent_t(streams->event_join) : nullptr));
}

sorf_status sorf_solve_f64_streamed(int32_t D, const double* G, const double* Zty, double lambda,
                                    int32_t n_refine, double* alpha, int32_t* info,
                                    void* workspace, size_t workspace_bytes,
                                    const sorf_solve_streams* streams, sorf_stream_t stream) {
  sorf_status s = check_solve(D, G, Zty, lambda, n_refine, alpha, info, workspace,
                              workspace_bytes);
  if (s != SORF_OK) return s;
  if ((s = check_streams(streams, stream)) != SORF_OK) return s;
  return dev(sorf_launch_solve_f64(D, G, Zty, lambda, n_refine, alpha, info, workspace,
                                   hipStream_t(stream),
                                   streams ? hipStream_t(streams->side) : nullptr,
                                   streams ? hipEvent_t(streams->event_fork) : nullptr,
                                   streams ? hipEvent_t(streams->event_join) : nullptr));
}

sorf_status sorf_solve(int32_t D, const float* G, const float* Zty, double lambda,
                       int32_t n_refine, double* alpha, int32_t* info, void* workspace,
                       size_t workspace_bytes, sorf_stream_t stream) {
  return sorf_solve_streamed(D, G, Zty, lambda, n_refine, alpha, info, workspace,
                             workspace_bytes, nullptr, stream);
}

sorf_status sorf_solve_f64(int32_t D, const double* G, const double* Zty, double lambda,
                           int32_t n_refine, double* alpha, int32_t* info, void* workspace,
                           size_t workspace_bytes, sorf_stream_t stream) {
  return sorf_solve_f64_streamed(D, G, Zty, lambda, n_refine, alpha, info, workspace,
                                 workspace_bytes, nullptr, stream);
}

size_t sorf_predict_workspace_bytes(const sorf_model* model, int64_t n_atoms, int64_t n_mols) {
  if (check_model(model) != SORF_OK || n_atoms < 0 || n_mols < 0) return 0;
  return predict_ws(model, n_atoms, n_mols);
}

}  // extern "C"

namespace {

sorf_status check_predict(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                          const float* J, const int64_t* J_ptr, const float* E, const float* F) {
  sorf_status s = check_model(model);
  if (s != SORF_OK) return s;
  if ((s = check_batch(batch)) != SORF_OK) return s;
  if ((J == nullptr) != (J_ptr == nullptr)) return SORF_ERR_INVALID_ARG;
  if ((J == nullptr) != (F == nullptr)) return SORF_ERR_INVALID_ARG;
  if (batch->n_mols > 0 && E == nullptr) return SORF_ERR_INVALID_ARG;
  if (batch->n_atoms > 0 && alpha == nullptr) return SORF_ERR_INVALID_ARG;
  if (!aligned16(alpha)) return SORF_ERR_INVALID_ARG;
  return SORF_OK;
}

// The launches of sorf_predict on a checked batch and a workspace of at least
// predict_ws() bytes, 256-byte aligned.
sorf_status predict_launch(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                           const float* J, const int64_t* J_ptr, float* E, float* F,
                           void* workspace, hipStream_t st) {
  const size_t need = predict_ws(model, batch->n_atoms, batch->n_mols);
  const SorfFeatureArgs a = pack(model, batch);
  if (J == nullptr) {
    // energies only: per (chunk of a molecule's atoms, stack) partials
    if (batch->n_atoms == 0) return dev(sorf_launch_fill(E, batch->n_mols, 0.0f, st));
    char* base = static_cast<char*>(workspace) + need -
                 energy_ws(model, batch->n_atoms, batch->n_mols);
    int64_t* chunk_ptr = reinterpret_cast<int64_t*>(base);
    float* part = reinterpret_cast<float*>(
        base + align256(sizeof(int64_t) * size_t(batch->n_mols + 1)));
    return dev(sorf_launch_energies(a, alpha, chunk_ptr, part, E, st));
  }
  float* e_atom = static_cast<float*>(workspace);
  const size_t grad_off = align256(sizeof(float) * size_t(batch->n_atoms));
  float* grad = reinterpret_cast<float*>(static_cast<char*>(workspace) + grad_off);
  void* plan = static_cast<char*>(workspace) + grad_off +
               align256(sizeof(float) * size_t(batch->n_atoms) * size_t(model->d));
  hipError_t e = sorf_launch_atom_adjoint(a, alpha, nullptr, J ? grad : nullptr, e_atom, st);
  if (e != hipSuccess) return SORF_ERR_DEVICE;
  return dev(sorf_launch_molecule_reduce(a, e_atom, grad, J, J_ptr, E, F, plan, st));
}

}  // namespace

extern "C" {

sorf_status sorf_predict(const sorf_model* model, const sorf_batch* batch, const float* alpha,
                         const float* J, const int64_t* J_ptr, float* E, float* F,
                         void* workspace, size_t workspace_bytes, sorf_stream_t stream) {
  sorf_status s = check_predict(model, batch, alpha, J, J_ptr, E, F);
  if (s != SORF_OK) return s;
  const size_t need = predict_ws(model, batch->n_atoms, batch->n_mols);
  if (batch->n_atoms > 0) {
    if (workspace == nullptr || workspace_bytes < need) return SORF_ERR_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  }
  return predict_launch(model, batch, alpha, J, J_ptr, E, F, workspace, hipStream_t(stream));
}

size_t sorf_forces_workspace_bytes(int64_t n_atoms, int64_t n_mols) {
  if (n_atoms < 0 || n_mols < 0) return 0;
  return sorf_force_plan_bytes(n_atoms, n_mols);
}

sorf_status sorf_forces(int32_t d, int64_t n_atoms, int64_t n_mols, const int64_t* mol_ptr,
                        const float* grad_x, const float* J, const int64_t* J_ptr, float* F,
                        void* workspace, size_t workspace_bytes, sorf_stream_t stream) {
  if (d < 1 || n_atoms < 0 || n_mols < 0 || mol_ptr == nullptr) return SORF_ERR_INVALID_ARG;
  if (n_atoms > (int64_t(1) << 40) || n_mols > (int64_t(1) << 31) - 1) return SORF_ERR_INVALID_ARG;
  if (n_atoms == 0) return SORF_OK;
  if (n_mols == 0) return SORF_ERR_INVALID_ARG;   // atoms need a molecule
  if (grad_x == nullptr || J == nullptr || J_ptr == nullptr || F == nullptr)
    return SORF_ERR_INVALID_ARG;
  if (workspace == nullptr || workspace_bytes < sorf_force_plan_bytes(n_atoms, n_mols))
    return SORF_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return SORF_ERR_WORKSPACE;
  SorfFeatureArgs a{};
  a.d = d;
  a.mol_ptr = mol_ptr;
  a.n_atoms = n_atoms;
  a.n_mols = n_mols;
  return dev(sorf_launch_molecule_reduce(a, nullptr, grad_x, J, J_ptr, nullptr, F, workspace,
                                         hipStream_t(stream)));
}

sorf_status sorf_validate_batch(const sorf_batch* batch, int32_t n_elements, int32_t* result,
                                sorf_stream_t stream) {
  sorf_status s = check_batch(batch);
  if (s != SORF_OK) return s;
  if (n_elements < 1 || result == nullptr) return SORF_ERR_INVALID_ARG;
  SorfFeatureArgs a{};
  a.element = batch->element;
  a.mol_ptr = batch->mol_ptr;
  a.n_atoms = batch->n_atoms;
  a.n_mols = batch->n_mols;
  a.n_elements = n_elements;
  return dev(sorf_launch_validate(a, result, hipStream_t(stream)));
}

}  // extern "C"

// ------------------------------------------------ sorf_predict_noalloc
// For callers that cannot allocate (graph capture, serving loops): the
// workspace of sorf_predict lives in a file-scope device array. Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in symbol); it passes the device address hipGetSymbolAddress returns
// for the current device, looked up once per device and kept.
namespace {

constexpr size_t kPredictScratchBytes = SORF_PREDICT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kPredictScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, or nullptr if the lookup failed.
void* scratch_for_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

sorf_status sorf_predict_noalloc(const sorf_model* model, const sorf_batch* batch,
                                 const float* alpha, const float* J, const int64_t* J_ptr,
                                 float* E, float* F, sorf_stream_t stream) {
  sorf_status s = check_predict(model, batch, alpha, J, J_ptr, E, F);
  if (s != SORF_OK) return s;
  if (predict_ws(model, batch->n_atoms, batch->n_mols) > kPredictScratchBytes)
    return SORF_ERR_WORKSPACE;
  void* ws = scratch_for_current_device();
  if (ws == nullptr) return SORF_ERR_DEVICE;
  return predict_launch(model, batch, alpha, J, J_ptr, E, F, ws, hipStream_t(stream));
}

}  // extern "C"
