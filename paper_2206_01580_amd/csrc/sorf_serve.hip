// Continuous-batching server for energy + force requests (C ABI).
//
// Paper: arXiv 2206.01580, Timings subsection (predicting many configurations
// in one call raises GPU utilisation by orders of magnitude over one small
// molecule at a time).
//
// The server keeps one persistent kernel resident on every compute unit
// (serve_kernel, cooperative launch). The host publishes batches of requests
// whose atoms are contiguous in a device-resident request pool: it writes a
// descriptor into a ring in host-coherent memory and advances the head count;
// the kernel takes the batches in order and writes each batch's energies and
// forces into the ring slot's host-coherent result area, then advances the
// done count. A batch therefore costs the host a descriptor write and no
// launch, copy or event; the device runs it without launch gaps.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>

#include "../../include/sorf.h"
#include "sorf_internal.h"

struct sorf_server {
  ServeKernelArgs args;
  ServeDesc* ring = nullptr;      // host-coherent
  ServeControl* ctl = nullptr;    // host-coherent
  float* results = nullptr;       // host-coherent
  hipStream_t stream = nullptr;
  int64_t ring_slots = 0, max_atoms = 0, submitted = 0;
  int32_t d = 0;
};

namespace {

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

bool serve_model_ok(const sorf_model* m) {
  return m != nullptr && m->d >= 2 && m->d <= 1024 && (m->d & (m->d - 1)) == 0 &&
         m->n_stacks >= 1 && m->n_elements >= 1 && m->n_transforms >= 1 &&
         m->n_transforms <= 3 && m->sigma > 0.0f && std::isfinite(m->sigma) &&
         int64_t(m->d) * m->n_stacks <= (int64_t(1) << 20) && m->signs != nullptr &&
         m->bias != nullptr;
}

bool serve_config_ok(const sorf_server_config* c) {
  return c != nullptr && c->max_batch_atoms >= 1 && c->max_batch_atoms <= (int64_t(1) << 24) &&
         c->ring_slots >= 1 && c->ring_slots <= 64 && c->idle_timeout_s > 0.0 &&
         c->idle_timeout_s <= 3600.0;
}

}  // namespace

extern "C" {

size_t sorf_server_workspace_bytes(const sorf_model* model, const sorf_server_config* cfg) {
  if (!serve_model_ok(model) || !serve_config_ok(cfg)) return 0;
  return sorf_serve_scratch_bytes(model->d, cfg->max_batch_atoms);
}

sorf_status sorf_server_start(const sorf_model* model, const float* alpha, const float* x_pool,
                              const int32_t* element_pool, const float* J_pool,
                              const sorf_server_config* cfg, void* workspace,
                              size_t workspace_bytes, sorf_stream_t stream, sorf_server** server) {
  if (server == nullptr) return SORF_ERR_INVALID_ARG;
  *server = nullptr;
  if (!serve_model_ok(model) || !serve_config_ok(cfg)) return SORF_ERR_INVALID_ARG;
  if (alpha == nullptr || x_pool == nullptr || element_pool == nullptr || J_pool == nullptr)
    return SORF_ERR_INVALID_ARG;
  const size_t need = sorf_serve_scratch_bytes(model->d, cfg->max_batch_atoms);
  if (workspace == nullptr || workspace_bytes < need ||
      (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
    return SORF_ERR_WORKSPACE;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return SORF_ERR_DEVICE;

  sorf_server* s = new (std::nothrow) sorf_server();
  if (s == nullptr) return SORF_ERR_DEVICE;
  s->ring_slots = cfg->ring_slots;
  s->max_atoms = cfg->max_batch_atoms;
  s->d = model->d;
  s->stream = hipStream_t(stream);
  const int64_t slot_floats = kServeMaxRequests + 3 * cfg->max_batch_atoms;
  const unsigned flags = hipHostMallocCoherent | hipHostMallocMapped;
  if (hipHostMalloc(reinterpret_cast<void**>(&s->ring), sizeof(ServeDesc) * size_t(s->ring_slots),
                    flags) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->ctl), sizeof(ServeControl), flags) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->results),
                    sizeof(float) * size_t(slot_floats) * size_t(s->ring_slots),
                    flags) != hipSuccess) {
    if (s->ring) (void)hipHostFree(s->ring);
    if (s->ctl) (void)hipHostFree(s->ctl);
    if (s->results) (void)hipHostFree(s->results);
    delete s;
    return SORF_ERR_DEVICE;
  }
  std::memset(s->ring, 0, sizeof(ServeDesc) * size_t(s->ring_slots));
  std::memset(s->ctl, 0, sizeof(ServeControl));

  // device scratch: [descriptor][barrier counters][grad][e_atom][partials]
  char* w = static_cast<char*>(workspace);
  ServeKernelArgs& a = s->args;
  a.d = model->d;
  a.n_stacks = model->n_stacks;
  a.n_transforms = model->n_transforms;
  a.n_waves = sorf_adjoint_waves(model->d, model->n_stacks);
  a.signs = model->signs;
  a.bias = model->bias;
  a.alpha = alpha;
  a.x_pool = x_pool;
  a.element_pool = element_pool;
  a.J_pool = J_pool;
  a.ring = s->ring;
  a.ctl = s->ctl;
  a.results = s->results;
  a.ring_slots = s->ring_slots;
  a.slot_floats = slot_floats;
  a.max_atoms = cfg->max_batch_atoms;
  a.dev_desc = reinterpret_cast<ServeDesc*>(w);
  w += al256(sizeof(ServeDesc));
  a.bar = reinterpret_cast<unsigned long long*>(w);
  w += al256(2 * sizeof(unsigned long long));
  a.grad = reinterpret_cast<float*>(w);
  w += al256(sizeof(float) * size_t(cfg->max_batch_atoms) * size_t(model->d));
  a.e_atom = reinterpret_cast<float*>(w);
  w += al256(sizeof(float) * size_t(cfg->max_batch_atoms));
  a.partial = reinterpret_cast<float*>(w);
  SorfFeatureArgs fa{};
  fa.d = model->d;
  fa.n_stacks = model->n_stacks;
  fa.n_transforms = model->n_transforms;
  fa.sigma = model->sigma;
  sorf_adjoint_scales(fa, &a.c_rev, &a.g_scale, &a.e_scale);
  // limits on the device's constant-rate counter (s_memrealtime)
  int clock_khz = 0;
  if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      clock_khz < 1)
    clock_khz = 100000;   // 100 MHz, the gfx9 real-time counter
  const double ticks_per_s = double(clock_khz) * 1e3;
  a.wait_ticks = int64_t(2.0 * ticks_per_s);                          // 2 s per phase
  a.idle_ticks = int64_t(cfg->idle_timeout_s * ticks_per_s) + 1;

  if (hipMemsetAsync(a.bar, 0, 2 * sizeof(unsigned long long), s->stream) != hipSuccess ||
      sorf_launch_serve(a, cus, s->stream) != hipSuccess) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipHostFree(s->ring);
    (void)hipHostFree(s->ctl);
    (void)hipHostFree(s->results);
    delete s;
    return SORF_ERR_DEVICE;
  }
  *server = s;
  return SORF_OK;
}

sorf_status sorf_server_submit(sorf_server* s, int32_t n_requests, const int64_t* atom_offsets,
                               const int64_t* J_offsets, int64_t* ticket) {
  if (s == nullptr || ticket == nullptr || atom_offsets == nullptr || J_offsets == nullptr)
    return SORF_ERR_INVALID_ARG;
  *ticket = -1;
  if (n_requests < 1 || n_requests > kServeMaxRequests) return SORF_ERR_INVALID_ARG;
  const int64_t n_atoms = atom_offsets[n_requests] - atom_offsets[0];
  if (atom_offsets[0] < 0 || n_atoms < 1 || n_atoms > s->max_atoms) return SORF_ERR_INVALID_ARG;
  for (int32_t r = 0; r < n_requests; ++r)
    if (atom_offsets[r + 1] < atom_offsets[r] || J_offsets[r] < 0) return SORF_ERR_INVALID_ARG;
  const int64_t done = __atomic_load_n(&s->ctl->done, __ATOMIC_ACQUIRE);
  if (s->submitted - done >= s->ring_slots) return SORF_ERR_BUSY;
  if (__atomic_load_n(&s->ctl->state, __ATOMIC_ACQUIRE) != 0) return SORF_ERR_DEVICE;

  const int64_t k = s->submitted;
  ServeDesc& dsc = s->ring[k % s->ring_slots];
  dsc.atom0 = atom_offsets[0];
  dsc.n_atoms = n_atoms;
  dsc.n_req = n_requests;
  dsc.slot = k % s->ring_slots;
  int64_t tiles = 0, parts = 0;
  for (int32_t r = 0; r < n_requests; ++r) {
    const int64_t n = atom_offsets[r + 1] - atom_offsets[r];
    dsc.mol_ptr[r] = atom_offsets[r] - atom_offsets[0];
    dsc.j_ptr[r] = J_offsets[r];
    dsc.tile_start[r] = tiles;
    dsc.part_start[r] = parts;
    const ForceShape f = force_shape(n, s->d);
    tiles += f.nrc * f.ncb;
    parts += f.nrc * 3 * n;
  }
  dsc.mol_ptr[n_requests] = n_atoms;
  dsc.j_ptr[n_requests] = 0;
  dsc.tile_start[n_requests] = tiles;
  dsc.part_start[n_requests] = parts;
  // the descriptor is complete before the head count that publishes it
  std::atomic_thread_fence(std::memory_order_release);
  __atomic_store_n(&s->ctl->head, k + 1, __ATOMIC_RELEASE);
  s->submitted = k + 1;
  *ticket = k;
  return SORF_OK;
}

int32_t sorf_server_query(const sorf_server* s, int64_t ticket) {
  if (s == nullptr || ticket < 0 || ticket >= s->submitted) return -2;
  if (__atomic_load_n(&s->ctl->done, __ATOMIC_ACQUIRE) > ticket) return 1;
  return __atomic_load_n(&s->ctl->state, __ATOMIC_ACQUIRE) != 0 ? -1 : 0;
}

const float* sorf_server_energies(const sorf_server* s, int64_t ticket) {
  if (s == nullptr || ticket < 0 || ticket >= s->submitted) return nullptr;
  return s->results + (ticket % s->ring_slots) * s->args.slot_floats;
}

const float* sorf_server_forces(const sorf_server* s, int64_t ticket) {
  const float* e = sorf_server_energies(s, ticket);
  return e == nullptr ? nullptr : e + kServeMaxRequests;
}

sorf_status sorf_server_stop(sorf_server* s, int32_t* state) {
  if (s == nullptr) return SORF_ERR_INVALID_ARG;
  __atomic_store_n(&s->ctl->stop, 1, __ATOMIC_RELEASE);
  const hipError_t e = hipStreamSynchronize(s->stream);
  if (state != nullptr) *state = __atomic_load_n(&s->ctl->state, __ATOMIC_ACQUIRE);
  (void)hipHostFree(s->ring);
  (void)hipHostFree(s->ctl);
  (void)hipHostFree(s->results);
  delete s;
  return e == hipSuccess ? SORF_OK : SORF_ERR_DEVICE;
}

}  // extern "C"
