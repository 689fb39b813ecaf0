// extern "C" boundary: argument checks, error translation, handles.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "codec.h"
#include "trace.h"

using namespace edpc;

struct edpc_model {
  std::unique_ptr<Model> m;
};
struct edpc_session {
  std::unique_ptr<Session> s;
};

namespace {
thread_local std::string g_last_error;

edpc_status set_err(edpc_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

template <class F>
edpc_status guarded(const char* name, F&& f) {
  TraceRange range(name);
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    return set_err(e.status, e.msg);
  } catch (const std::bad_alloc&) {
    return set_err(EDPC_E_NOMEM, "host allocation failed");
  } catch (...) {
    return set_err(EDPC_E_DEVICE, "unexpected internal error");
  }
}

hipStream_t S(void* p) { return (hipStream_t)p; }
}  // namespace

extern "C" {

const char* edpc_status_string(int st) {
  switch (st) {
    case EDPC_OK: return "ok";
    case EDPC_E_INVALID_ARG: return "invalid argument";
    case EDPC_E_NOMEM: return "out of memory";
    case EDPC_E_CAPACITY: return "output buffer too small";
    case EDPC_E_CORRUPT: return "corrupt or truncated container";
    case EDPC_E_CHECKSUM: return "checksum mismatch";
    case EDPC_E_UNSUPPORTED: return "unsupported format, device or kernel configuration";
    case EDPC_E_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* edpc_last_error(void) { return g_last_error.c_str(); }
int edpc_abi_version(void) { return EDPC_ABI_VERSION; }

edpc_status edpc_config_default(edpc_config* cfg) {
  if (!cfg) return set_err(EDPC_E_INVALID_ARG, "cfg is NULL");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->struct_size = sizeof(edpc_config);
  cfg->context = 16;
  cfg->embed = 16;
  cfg->latent = 64;
  cfg->blocks = 2;
  cfg->hidden = 128;
  cfg->branches = 2;
  cfg->cdf_bits = 16;
  cfg->precision = EDPC_FP32;
  cfg->flags = 0;
  cfg->lr = 1e-3f;
  cfg->beta1 = 0.9f;
  cfg->beta2 = 0.999f;
  cfg->eps = 1e-8f;
  cfg->seed = 0;
  return EDPC_OK;
}

edpc_status edpc_config_validate(const edpc_config* cfg) {
  return guarded("edpc_config_validate", [&] {
    if (!cfg) fail(EDPC_E_INVALID_ARG, "cfg is NULL");
    Model::validate(*cfg);
    return EDPC_OK;
  });
}

edpc_status edpc_encode_bound(const edpc_config* cfg, const uint64_t* h_lens, size_t n,
                              size_t* bound) {
  return guarded("edpc_encode_bound", [&] {
    if (!cfg || !bound || (n && !h_lens)) fail(EDPC_E_INVALID_ARG, "NULL argument");
    Model::validate(*cfg);
    if (n == 0) fail(EDPC_E_INVALID_ARG, "n_streams must be >= 1");
    *bound = encode_bound(*cfg, h_lens, n);
    return EDPC_OK;
  });
}

edpc_status edpc_encoder_begin(const edpc_config* cfg, const uint8_t* d_in, const uint64_t* h_lens,
                               size_t n, void* stream, edpc_session** out) {
  return guarded("edpc_encoder_begin", [&] {
    if (!cfg || !out || !h_lens) fail(EDPC_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    uint64_t total = 0;
    for (size_t i = 0; i < n; ++i) total += h_lens[i];
    if (total && !d_in) fail(EDPC_E_INVALID_ARG, "d_in is NULL");
    std::unique_ptr<edpc_session> h(new edpc_session());
    h->s = encoder_begin(*cfg, d_in, h_lens, n, S(stream), nullptr);
    *out = h.release();
    return EDPC_OK;
  });
}

edpc_status edpc_decoder_begin(const uint8_t* d_in, size_t in_len, uint8_t* d_out, size_t out_cap,
                               void* stream, edpc_session** out) {
  return guarded("edpc_decoder_begin", [&] {
    if (!d_in || !out) fail(EDPC_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    std::unique_ptr<edpc_session> h(new edpc_session());
    h->s = decoder_begin(d_in, in_len, d_out, out_cap, S(stream));
    *out = h.release();
    return EDPC_OK;
  });
}

edpc_status edpc_session_run(edpc_session* s, uint64_t n_steps, uint64_t* done) {
  return guarded("edpc_session_run", [&] {
    if (!s || !s->s) fail(EDPC_E_INVALID_ARG, "NULL session");
    const uint64_t before = s->s->next;
    s->s->run(n_steps);
    if (done) *done = s->s->next - before;
    return EDPC_OK;
  });
}

edpc_status edpc_session_progress(const edpc_session* s, uint64_t* step, uint64_t* total) {
  if (!s || !s->s) return set_err(EDPC_E_INVALID_ARG, "NULL session");
  if (step) *step = s->s->next;
  if (total) *total = s->s->maxlen;
  return EDPC_OK;
}

edpc_status edpc_encoder_finish(edpc_session* s, uint8_t* d_out, size_t out_cap, size_t* out_len) {
  return guarded("edpc_encoder_finish", [&] {
    if (!s || !s->s || s->s->decoding) fail(EDPC_E_INVALID_ARG, "not an encoder session");
    if (!out_len) fail(EDPC_E_INVALID_ARG, "out_len is NULL");
    try {
      *out_len = encoder_finish(*s->s, d_out, out_cap);
    } catch (const Error& e) {
      if (e.status == EDPC_E_CAPACITY) *out_len = s->s->out_cap;
      throw;
    }
    return EDPC_OK;
  });
}

edpc_status edpc_decoder_finish(edpc_session* s, size_t* out_len) {
  return guarded("edpc_decoder_finish", [&] {
    if (!s || !s->s || !s->s->decoding) fail(EDPC_E_INVALID_ARG, "not a decoder session");
    const size_t n = decoder_finish(*s->s);
    if (out_len) *out_len = n;
    return EDPC_OK;
  });
}

void edpc_session_destroy(edpc_session* s) { delete s; }

edpc_status edpc_session_time_kernels(edpc_session* s, uint64_t n_steps, float* h_ms,
                                      uint32_t* h_launches) {
  return guarded("edpc_session_time_kernels", [&] {
    if (!s || !s->s || !h_ms || !h_launches) fail(EDPC_E_INVALID_ARG, "NULL argument");
    KTimer timer;
    Model& m = *s->s->model;
    m.timer = &timer;
    try {
      s->s->run(n_steps);
      timer.collect(h_ms, h_launches);
    } catch (...) {
      m.timer = nullptr;
      throw;
    }
    m.timer = nullptr;
    return EDPC_OK;
  });
}

const char* edpc_kclass_name(int c) { return kclass_name(c); }

edpc_status edpc_encode(const edpc_config* cfg, const uint8_t* d_in, const uint64_t* h_lens,
                        size_t n, uint8_t* d_out, size_t out_cap, size_t* out_len, void* stream) {
  edpc_session* s = nullptr;
  edpc_status st = edpc_encoder_begin(cfg, d_in, h_lens, n, stream, &s);
  if (st != EDPC_OK) return st;
  st = edpc_encoder_finish(s, d_out, out_cap, out_len);
  std::string keep = g_last_error;
  edpc_session_destroy(s);
  g_last_error = keep;
  return st;
}

edpc_status edpc_decode(const uint8_t* d_in, size_t in_len, uint8_t* d_out, size_t out_cap,
                        size_t* out_len, void* stream) {
  edpc_session* s = nullptr;
  edpc_status st = edpc_decoder_begin(d_in, in_len, d_out, out_cap, stream, &s);
  if (st != EDPC_OK) return st;
  st = edpc_decoder_finish(s, out_len);
  std::string keep = g_last_error;
  edpc_session_destroy(s);
  g_last_error = keep;
  return st;
}

edpc_status edpc_encode_host(const edpc_config* cfg, const uint8_t* h_in, const uint64_t* h_lens,
                             size_t n, uint8_t* h_out, size_t out_cap, size_t* out_len,
                             uint32_t chunk_steps, void* stream) {
  return guarded("edpc_encode_host", [&] {
    if (!cfg || !h_lens || !out_len || !h_out) fail(EDPC_E_INVALID_ARG, "NULL argument");
    uint64_t total = 0;
    for (size_t i = 0; i < n; ++i) total += h_lens[i];
    if (total && !h_in) fail(EDPC_E_INVALID_ARG, "h_in is NULL");
    size_t need = 0;
    try {
      *out_len = stream_encode(*cfg, h_in, h_lens, n, h_out, out_cap, chunk_steps, S(stream), &need);
    } catch (const Error& e) {
      if (e.status == EDPC_E_CAPACITY) *out_len = need;
      throw;
    }
    return EDPC_OK;
  });
}

edpc_status edpc_decode_host(const uint8_t* h_in, size_t in_len, uint8_t* h_out, size_t out_cap,
                             size_t* out_len, uint32_t chunk_steps, void* stream) {
  return guarded("edpc_decode_host", [&] {
    if (!h_in || !out_len) fail(EDPC_E_INVALID_ARG, "NULL argument");
    if (!h_out && out_cap) fail(EDPC_E_INVALID_ARG, "h_out is NULL");
    *out_len = stream_decode(h_in, in_len, h_out, out_cap, chunk_steps, S(stream));
    return EDPC_OK;
  });
}

edpc_status edpc_decode_info(const uint8_t* h_in, size_t in_len, edpc_config* cfg,
                             size_t* n_streams, uint64_t* h_lens, size_t lens_cap,
                             size_t* header_len, size_t* decoded_len) {
  return guarded("edpc_decode_info", [&] {
    if (!h_in) fail(EDPC_E_INVALID_ARG, "h_in is NULL");
    Header h;
    size_t need = 0;
    std::string err;
    const edpc_status st = parse_header(h_in, in_len, &h, &need, &err);
    if (header_len) *header_len = need;
    if (st != EDPC_OK) fail(st, err);
    if (cfg) *cfg = h.cfg;
    if (n_streams) *n_streams = h.lens.size();
    if (h_lens) {
      if (lens_cap < h.lens.size()) fail(EDPC_E_CAPACITY, "lens_cap smaller than n_streams");
      std::memcpy(h_lens, h.lens.data(), h.lens.size() * 8);
    }
    if (decoded_len) {
      size_t t = 0;
      for (uint64_t l : h.lens) t += l;
      *decoded_len = t;
    }
    return EDPC_OK;
  });
}

// ---------------------------------------------------------------- model

edpc_status edpc_model_create(const edpc_config* cfg, size_t n_slots, size_t max_rows,
                              edpc_model** out) {
  return guarded("edpc_model_create", [&] {
    if (!cfg || !out) fail(EDPC_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    std::unique_ptr<edpc_model> h(new edpc_model());
    h->m.reset(new Model(*cfg, n_slots, max_rows, nullptr));
    h->m->init_params(nullptr);
    h->m->build_tables(nullptr);
    if (cfg->flags & EDPC_CFG_AUTOTUNE) h->m->autotune(nullptr);
    hip_check(hipDeviceSynchronize(), "model create");
    *out = h.release();
    return EDPC_OK;
  });
}

edpc_status edpc_model_create_with_kernels(const edpc_config* cfg, size_t n_slots,
                                           size_t max_rows, uint64_t kernel_id,
                                           edpc_model** out) {
  return guarded("edpc_model_create_with_kernels", [&] {
    if (!cfg || !out) fail(EDPC_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (kernel_id == 0) return edpc_model_create(cfg, n_slots, max_rows, out);
    KernelConfig kc;
    if (!KernelConfig::decode(kernel_id, &kc)) fail(EDPC_E_UNSUPPORTED, "unknown kernel configuration");
    Model::validate(*cfg);
    const bool bf16 = cfg->precision == EDPC_BF16;
    for (int ps = 0; ps < PS_COUNT; ++ps) {
      const EpiKind epi = ps == PS_GATE ? EPI_GATE_FWD : ps == PS_GATE_BWD ? EPI_GATE_BWD : EPI_STORE;
      const int nb = ps == PS_GATE ? (int)cfg->branches : 1;
      if (!wide_tile_supported(kc.tile[ps], bf16, epi, nb))
        fail(EDPC_E_UNSUPPORTED, "tile of the kernel configuration does not serve this model");
    }
    std::unique_ptr<edpc_model> h(new edpc_model());
    h->m.reset(new Model(*cfg, n_slots, max_rows, &kc));
    h->m->init_params(nullptr);
    h->m->build_tables(nullptr);
    hip_check(hipDeviceSynchronize(), "model create");
    *out = h.release();
    return EDPC_OK;
  });
}

edpc_status edpc_model_kernel_id(const edpc_model* mh, uint64_t* kernel_id) {
  if (!mh || !mh->m || !kernel_id) return set_err(EDPC_E_INVALID_ARG, "NULL argument");
  *kernel_id = mh->m->kc.encode();
  return EDPC_OK;
}

void edpc_model_destroy(edpc_model* m) {
  if (m) (void)hipDeviceSynchronize();
  delete m;
}

edpc_status edpc_model_step(edpc_model* mh, const uint8_t* d_ctx, const uint8_t* d_target,
                            const uint32_t* h_slot, size_t rows, float* d_probs, uint32_t* d_cum,
                            float* d_loss, uint32_t flags, void* stream) {
  return guarded("edpc_model_step", [&] {
    if (!mh || !mh->m) fail(EDPC_E_INVALID_ARG, "NULL model");
    Model& m = *mh->m;
    if (flags & ~(EDPC_STEP_BACKWARD | EDPC_STEP_UPDATE | EDPC_STEP_KEEP_FDM_GRAD))
      fail(EDPC_E_INVALID_ARG, "unknown step flags");
    if (rows == 0 || rows > m.max_rows) fail(EDPC_E_INVALID_ARG, "rows must be in 1..max_rows");
    if (!d_ctx || !h_slot) fail(EDPC_E_INVALID_ARG, "d_ctx and h_slot are required");
    const bool bwd = flags != 0;
    if ((bwd || d_loss) && !d_target) fail(EDPC_E_INVALID_ARG, "d_target is required for the loss and gradients");
    std::vector<char> seen(m.n_slots, 0);
    for (size_t r = 0; r < rows; ++r) {
      if (h_slot[r] >= m.n_slots) fail(EDPC_E_INVALID_ARG, "slot index out of range");
      if (seen[h_slot[r]]) fail(EDPC_E_INVALID_ARG, "slot indices must be distinct");
      seen[h_slot[r]] = 1;
    }
    hipStream_t s = S(stream);
    hip_check(hipMemcpyAsync(m.ctx, d_ctx, rows * m.C, hipMemcpyDeviceToDevice, s), "copy");
    if (d_target) hip_check(hipMemcpyAsync(m.tgt, d_target, rows, hipMemcpyDeviceToDevice, s), "copy");
    hip_check(hipMemcpyAsync(m.slot, h_slot, rows * sizeof(uint32_t), hipMemcpyHostToDevice, s), "copy");
    StepOutputs out;
    out.probs = d_probs;
    out.cum = d_cum;
    out.loss = d_loss;
    out.update = (flags & EDPC_STEP_UPDATE) != 0;
    out.backward = bwd;
    out.keep_fdm_grad = (flags & EDPC_STEP_KEEP_FDM_GRAD) != 0 && !out.update;
    if (out.keep_fdm_grad && !m.dUkeep) {
      void* p = nullptr;
      hip_check(hipMalloc(&p, m.n_slots * (size_t)m.L * m.L * sizeof(float)), "hipMalloc");
      m.allocs.push_back(p);
      m.dUkeep = (float*)p;
    }
    if (out.keep_fdm_grad)  // slots outside this call get a zero gradient
      hip_check(hipMemsetAsync(m.dUkeep, 0, m.n_slots * (size_t)m.L * m.L * sizeof(float), s), "memset");
    const uint32_t tau = out.update ? (uint32_t)(m.tau + 1) : (uint32_t)(m.tau > 0 ? m.tau : 1);
    k_step_explicit(m.st, (int)rows, tau, m.cfg.beta1, m.cfg.beta2, s);
    StreamIO io;
    std::memset(&io, 0, sizeof(io));
    io.slot = m.slot;
    out.has_target = d_target != nullptr;
    m.step(MODE_PLAIN, io, out, (int)rows, s);
    if (out.update) m.tau += 1;
    return EDPC_OK;
  });
}

edpc_status edpc_model_tensor_count(const edpc_model* mh, size_t* n) {
  if (!mh || !n) return set_err(EDPC_E_INVALID_ARG, "NULL argument");
  *n = mh->m->tens.size() + (mh->m->low_rank ? 3 : 1);
  return EDPC_OK;
}

edpc_status edpc_model_tensor_info(const edpc_model* mh, size_t idx, char* name, size_t cap,
                                   size_t* numel) {
  if (!mh) return set_err(EDPC_E_INVALID_ARG, "NULL model");
  const Model& m = *mh->m;
  std::string nm;
  size_t ne;
  if (idx < m.tens.size()) {
    nm = m.tens[idx].name;
    ne = m.tens[idx].numel;
  } else if (idx == m.tens.size()) {
    nm = "U";
    ne = m.n_slots * (size_t)m.L * m.L;
  } else if (m.low_rank && idx <= m.tens.size() + 2) {
    nm = idx == m.tens.size() + 1 ? "A" : "B";
    ne = m.n_slots * (size_t)m.F * m.L;
  } else {
    return set_err(EDPC_E_INVALID_ARG, "tensor index out of range");
  }
  if (name && cap) {
    std::strncpy(name, nm.c_str(), cap - 1);
    name[cap - 1] = 0;
  }
  if (numel) *numel = ne;
  return EDPC_OK;
}

static float* tensor_ptr(Model& m, uint32_t kind, size_t idx, size_t* numel, bool for_write) {
  if (idx < m.tens.size()) {
    const TensorInfo& t = m.tens[idx];
    *numel = t.numel;
    float* base = kind == EDPC_KIND_PARAM ? m.param : kind == EDPC_KIND_GRAD ? m.grad
                  : kind == EDPC_KIND_ADAM_M ? m.m : kind == EDPC_KIND_ADAM_V ? m.v : nullptr;
    if (!base) fail(EDPC_E_INVALID_ARG, "unknown tensor kind");
    return base + t.off;
  }
  if (idx == m.tens.size()) {
    *numel = m.n_slots * (size_t)m.L * m.L;
    if (kind == EDPC_KIND_PARAM) return m.U;
    if (kind == EDPC_KIND_ADAM_M) return m.mU;
    if (kind == EDPC_KIND_ADAM_V) return m.vU;
    if (kind == EDPC_KIND_GRAD) {
      if (!m.dUkeep) fail(EDPC_E_INVALID_ARG, "no FDM gradient kept (use EDPC_STEP_KEEP_FDM_GRAD)");
      if (for_write) fail(EDPC_E_INVALID_ARG, "the FDM gradient is read-only");
      return m.dUkeep;
    }
    fail(EDPC_E_INVALID_ARG, "unknown tensor kind");
  }
  if (m.low_rank && idx <= m.tens.size() + 2) {
    const bool a = idx == m.tens.size() + 1;
    *numel = m.n_slots * (size_t)m.F * m.L;
    if (kind == EDPC_KIND_PARAM) return a ? m.A : m.B;
    if (kind == EDPC_KIND_ADAM_M) return a ? m.mA : m.mB;
    if (kind == EDPC_KIND_ADAM_V) return a ? m.vA : m.vB;
    if (kind == EDPC_KIND_GRAD) fail(EDPC_E_INVALID_ARG, "the low-rank factor gradients are not kept");
    fail(EDPC_E_INVALID_ARG, "unknown tensor kind");
  }
  fail(EDPC_E_INVALID_ARG, "tensor index out of range");
}

}  // extern "C"

namespace {
float bf16_widen(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// The BF16 operand copy of shared tensor idx, widened, in its own layout.
void read_operand(Model& m, uint32_t kind, size_t idx, float* h_dst, size_t numel) {
  if (!m.bf16) fail(EDPC_E_INVALID_ARG, "FP32 models keep no operand copies");
  if (idx >= m.tens.size()) fail(EDPC_E_INVALID_ARG, "only shared tensors have operand copies");
  const TensorInfo& t = m.tens[idx];
  if (numel != t.numel) fail(EDPC_E_INVALID_ARG, "numel mismatch");
  hip_check(hipDeviceSynchronize(), "sync");
  if (!m.kc.fused) {
    std::vector<uint16_t> h(t.numel);
    hip_check(hipMemcpy(h.data(), m.p16 + t.off, t.numel * 2, hipMemcpyDeviceToHost), "copy");
    for (size_t i = 0; i < t.numel; ++i) h_dst[i] = bf16_widen(h[i]);
    return;
  }
  for (const Model::FragMat& fm : m.frag_mats) {
    const size_t size = (size_t)fm.rows * fm.cols;
    if (t.off < fm.off || t.off >= fm.off + size) continue;
    // the tensor is rows [r0, r0 + numel / cols) of the matrix
    const size_t r0 = (t.off - fm.off) / fm.cols, nrow = t.numel / fm.cols;
    std::vector<uint16_t> f(size);
    const uint4* src = kind == EDPC_KIND_OPERAND_NT ? fm.nt : fm.nn;
    hip_check(hipMemcpy(f.data(), src, size * 2, hipMemcpyDeviceToHost), "copy");
    // fragment (nb, kb) of KB k-blocks, lane l, element v (layouts in fused.h)
    for (size_t q = 0; q < size; ++q) {
      const size_t frag = q / 512, l = (q / 8) % 64, v = q % 8;
      size_t r, c;
      if (kind == EDPC_KIND_OPERAND_NT) {
        const size_t KB = fm.cols / 32, nb = frag / KB, kb = frag % KB;
        r = nb * 16 + l % 16;
        c = kb * 32 + 8 * (l / 16) + v;
      } else {
        const size_t KB = fm.rows / 32, nb = frag / KB, kb = frag % KB;
        r = kb * 32 + 8 * (l / 16) + v;
        c = nb * 16 + l % 16;
      }
      if (r >= r0 && r < r0 + nrow) h_dst[(r - r0) * fm.cols + c] = bf16_widen(f[q]);
    }
    return;
  }
  fail(EDPC_E_INVALID_ARG, "tensor " + t.name + " has no operand copy in the fused step");
}
}  // namespace

extern "C" {

edpc_status edpc_model_read(const edpc_model* mh, uint32_t kind, size_t idx, float* h_dst,
                            size_t numel) {
  return guarded("edpc_model_read", [&] {
    if (!mh || !h_dst) fail(EDPC_E_INVALID_ARG, "NULL argument");
    if (kind == EDPC_KIND_OPERAND_NT || kind == EDPC_KIND_OPERAND_NN) {
      read_operand(*mh->m, kind, idx, h_dst, numel);
      return EDPC_OK;
    }
    size_t ne = 0;
    float* p = tensor_ptr(*mh->m, kind, idx, &ne, false);
    if (numel != ne) fail(EDPC_E_INVALID_ARG, "numel mismatch");
    hip_check(hipDeviceSynchronize(), "sync");
    hip_check(hipMemcpy(h_dst, p, ne * sizeof(float), hipMemcpyDeviceToHost), "copy");
    return EDPC_OK;
  });
}

edpc_status edpc_model_write(edpc_model* mh, uint32_t kind, size_t idx, const float* h_src,
                             size_t numel) {
  return guarded("edpc_model_write", [&] {
    if (!mh || !h_src) fail(EDPC_E_INVALID_ARG, "NULL argument");
    Model& m = *mh->m;
    size_t ne = 0;
    float* p = tensor_ptr(m, kind, idx, &ne, true);
    if (numel != ne) fail(EDPC_E_INVALID_ARG, "numel mismatch");
    hip_check(hipDeviceSynchronize(), "sync");
    hip_check(hipMemcpy(p, h_src, ne * sizeof(float), hipMemcpyHostToDevice), "copy");
    if (kind == EDPC_KIND_PARAM && m.bf16 && idx < m.tens.size()) {
      const TensorInfo& t = m.tens[idx];
      k_to_bf16(m.param + t.off, m.p16 + t.off, t.numel, nullptr);
      if (m.kc.fused) m.build_frags(nullptr);
      hip_check(hipDeviceSynchronize(), "sync");
    }
    return EDPC_OK;
  });
}

edpc_status edpc_model_read_device(const edpc_model* mh, uint32_t kind, size_t idx, float* d_dst,
                                   size_t numel, void* stream) {
  return guarded("edpc_model_read_device", [&] {
    if (!mh || !d_dst) fail(EDPC_E_INVALID_ARG, "NULL argument");
    size_t ne = 0;
    float* p = tensor_ptr(*mh->m, kind, idx, &ne, false);
    if (numel != ne) fail(EDPC_E_INVALID_ARG, "numel mismatch");
    hip_check(hipMemcpyAsync(d_dst, p, ne * sizeof(float), hipMemcpyDeviceToDevice, S(stream)), "copy");
    return EDPC_OK;
  });
}

edpc_status edpc_model_write_device(edpc_model* mh, uint32_t kind, size_t idx, const float* d_src,
                                    size_t numel, void* stream) {
  return guarded("edpc_model_write_device", [&] {
    if (!mh || !d_src) fail(EDPC_E_INVALID_ARG, "NULL argument");
    Model& m = *mh->m;
    size_t ne = 0;
    float* p = tensor_ptr(m, kind, idx, &ne, true);
    if (numel != ne) fail(EDPC_E_INVALID_ARG, "numel mismatch");
    hip_check(hipMemcpyAsync(p, d_src, ne * sizeof(float), hipMemcpyDeviceToDevice, S(stream)), "copy");
    if (kind == EDPC_KIND_PARAM && m.bf16 && idx < m.tens.size()) {
      const TensorInfo& t = m.tens[idx];
      k_to_bf16(m.param + t.off, m.p16 + t.off, t.numel, S(stream));
      if (m.kc.fused) m.build_frags(S(stream));
    }
    return EDPC_OK;
  });
}

edpc_status edpc_model_activation(const edpc_model* mh, uint32_t block, float* d_dst, size_t numel,
                                  void* stream) {
  return guarded("edpc_model_activation", [&] {
    if (!mh || !mh->m || !d_dst) fail(EDPC_E_INVALID_ARG, "NULL argument");
    const Model& m = *mh->m;
    if (block > (uint32_t)m.N) fail(EDPC_E_INVALID_ARG, "block index out of range");
    if (m.last_rows == 0) fail(EDPC_E_INVALID_ARG, "no step has run");
    const float* src = m.block_input((int)block);
    if (!src) fail(EDPC_E_UNSUPPORTED, "the row-block step keeps no FP32 copy of the head's input");
    if (numel != (size_t)m.last_rows * m.F) fail(EDPC_E_INVALID_ARG, "numel must be rows * context * embed");
    hip_check(hipMemcpyAsync(d_dst, src, numel * sizeof(float), hipMemcpyDeviceToDevice, S(stream)),
              "copy");
    return EDPC_OK;
  });
}

edpc_status edpc_mutual_info(const float* d_z, size_t dz, const float* d_y, size_t dy, size_t c,
                             uint32_t v, double* h_mi, int32_t* d_counts, float* d_eps,
                             void* stream) {
  return guarded("edpc_mutual_info", [&] {
    if (!d_z || !d_y || !h_mi) fail(EDPC_E_INVALID_ARG, "NULL argument");
    *h_mi = mutual_info(d_z, dz, d_y, dy, c, v, d_counts, d_eps, S(stream));
    return EDPC_OK;
  });
}

edpc_status edpc_model_get_step(const edpc_model* mh, uint64_t* tau) {
  if (!mh || !tau) return set_err(EDPC_E_INVALID_ARG, "NULL argument");
  *tau = mh->m->tau;
  return EDPC_OK;
}

edpc_status edpc_model_set_step(edpc_model* mh, uint64_t tau) {
  if (!mh) return set_err(EDPC_E_INVALID_ARG, "NULL model");
  mh->m->tau = tau;
  return EDPC_OK;
}

// ---------------------------------------------------------------- whole state

}  // extern "C"

namespace {
struct BlobWriter {
  uint8_t* p;
  size_t cap, n = 0;
  void put(const void* src, size_t k) {
    if (p && n + k <= cap) std::memcpy(p + n, src, k);
    n += k;
  }
  void u32(uint32_t v) { put(&v, 4); }
  void u64(uint64_t v) { put(&v, 8); }
};
struct BlobReader {
  const uint8_t* p;
  size_t len, n = 0;
  const uint8_t* take(size_t k) {
    if (k > len - n) fail(EDPC_E_INVALID_ARG, "state blob truncated");
    const uint8_t* q = p + n;
    n += k;
    return q;
  }
  uint32_t u32() { uint32_t v; std::memcpy(&v, take(4), 4); return v; }
  uint64_t u64() { uint64_t v; std::memcpy(&v, take(8), 8); return v; }
};
constexpr uint32_t kStateVersion = 1;

void cfg_words(const edpc_config& c, uint32_t w[9]) {
  const uint32_t v[9] = {c.context, c.embed, c.latent, c.blocks, c.hidden, c.branches,
                         c.cdf_bits, c.precision, c.flags};
  std::memcpy(w, v, sizeof(v));
}

size_t n_tensors(const Model& m) { return m.tens.size() + (m.low_rank ? 3 : 1); }
std::string tensor_name(const Model& m, size_t i) {
  if (i < m.tens.size()) return m.tens[i].name;
  if (i == m.tens.size()) return "U";
  return i == m.tens.size() + 1 ? "A" : "B";
}
}  // namespace

extern "C" {

edpc_status edpc_model_get_state(const edpc_model* mh, void* h_buf, size_t cap, size_t* len) {
  return guarded("edpc_model_get_state", [&] {
    if (!mh || !mh->m || !len) fail(EDPC_E_INVALID_ARG, "NULL argument");
    Model& m = *mh->m;
    // size first: the blob is written only when it fits
    BlobWriter sz{nullptr, 0};
    const size_t nt = n_tensors(m);
    sz.n = 4 + 4 + 4 + 4 + 8 + 9 * 4 + 8;
    for (size_t i = 0; i < nt; ++i) {
      size_t ne = 0;
      (void)tensor_ptr(m, EDPC_KIND_PARAM, i, &ne, false);
      sz.n += 4 + ((tensor_name(m, i).size() + 3) & ~(size_t)3) + 8 + 3 * ne * sizeof(float);
    }
    *len = sz.n;
    if (!h_buf || cap < sz.n) fail(EDPC_E_CAPACITY, "state buffer too small");
    hip_check(hipDeviceSynchronize(), "sync");
    BlobWriter w{(uint8_t*)h_buf, cap};
    w.put("EDPS", 4);
    w.u32(kStateVersion);
    w.u32((uint32_t)nt);
    w.u32(0);
    w.u64(m.tau);
    uint32_t cw[9];
    cfg_words(m.cfg, cw);
    for (uint32_t v : cw) w.u32(v);
    w.u64(m.n_slots);
    for (size_t i = 0; i < nt; ++i) {
      const std::string nm = tensor_name(m, i);
      w.u32((uint32_t)nm.size());
      const size_t padded = (nm.size() + 3) & ~(size_t)3;
      std::string pad = nm;
      pad.resize(padded, '\0');
      w.put(pad.data(), padded);
      size_t ne = 0;
      (void)tensor_ptr(m, EDPC_KIND_PARAM, i, &ne, false);
      w.u64(ne);
      for (uint32_t kind : {EDPC_KIND_PARAM, EDPC_KIND_ADAM_M, EDPC_KIND_ADAM_V}) {
        const float* src = tensor_ptr(m, kind, i, &ne, false);
        hip_check(hipMemcpy((uint8_t*)h_buf + w.n, src, ne * sizeof(float), hipMemcpyDeviceToHost),
                  "copy");
        w.n += ne * sizeof(float);
      }
    }
    return EDPC_OK;
  });
}

edpc_status edpc_model_set_state(edpc_model* mh, const void* h_buf, size_t len) {
  return guarded("edpc_model_set_state", [&] {
    if (!mh || !mh->m || !h_buf) fail(EDPC_E_INVALID_ARG, "NULL argument");
    Model& m = *mh->m;
    BlobReader r{(const uint8_t*)h_buf, len};
    if (std::memcmp(r.take(4), "EDPS", 4) != 0) fail(EDPC_E_INVALID_ARG, "not a state blob");
    if (r.u32() != kStateVersion) fail(EDPC_E_INVALID_ARG, "state blob version");
    const uint32_t nt = r.u32();
    (void)r.u32();
    const uint64_t tau = r.u64();
    uint32_t cw[9];
    cfg_words(m.cfg, cw);
    for (uint32_t v : cw)
      if (r.u32() != v) fail(EDPC_E_INVALID_ARG, "state blob of another model configuration");
    if (r.u64() != m.n_slots) fail(EDPC_E_INVALID_ARG, "state blob of another slot count");
    if (nt != n_tensors(m)) fail(EDPC_E_INVALID_ARG, "state blob tensor count");
    // validate the whole blob before writing anything
    struct Part { size_t idx; const uint8_t* data; size_t ne; };
    std::vector<Part> parts;
    for (size_t i = 0; i < nt; ++i) {
      const uint32_t nl = r.u32();
      const uint8_t* nm = r.take((nl + 3) & ~(uint32_t)3);
      if (std::string((const char*)nm, nl) != tensor_name(m, i))
        fail(EDPC_E_INVALID_ARG, "state blob tensor name");
      size_t ne = 0;
      (void)tensor_ptr(m, EDPC_KIND_PARAM, i, &ne, false);
      if (r.u64() != ne) fail(EDPC_E_INVALID_ARG, "state blob tensor size");
      if (ne > (len - r.n) / (3 * sizeof(float))) fail(EDPC_E_INVALID_ARG, "state blob truncated");
      parts.push_back(Part{i, r.take(3 * ne * sizeof(float)), ne});
    }
    if (r.n != len) fail(EDPC_E_INVALID_ARG, "state blob has trailing bytes");
    hip_check(hipDeviceSynchronize(), "sync");
    for (const Part& pt : parts) {
      int q = 0;
      for (uint32_t kind : {EDPC_KIND_PARAM, EDPC_KIND_ADAM_M, EDPC_KIND_ADAM_V}) {
        size_t ne = 0;
        float* dst = tensor_ptr(m, kind, pt.idx, &ne, true);
        hip_check(hipMemcpy(dst, pt.data + (size_t)q * ne * sizeof(float), ne * sizeof(float),
                            hipMemcpyHostToDevice), "copy");
        ++q;
      }
    }
    if (m.bf16) {  // operand copies of the products follow the FP32 master
      k_to_bf16(m.param, m.p16, m.P, nullptr);
      if (m.kc.fused) m.build_frags(nullptr);
    }
    hip_check(hipDeviceSynchronize(), "sync");
    m.tau = tau;
    return EDPC_OK;
  });
}

// ---------------------------------------------------------------- coder only

edpc_status edpc_rc_encode(const uint32_t* d_cum, const uint8_t* d_sym, size_t n_steps,
                           size_t n_streams, uint8_t* d_out, size_t cap, uint32_t* h_out_lens,
                           void* stream) {
  return guarded("edpc_rc_encode", [&] {
    if (!d_cum || !d_sym || !d_out || !h_out_lens) fail(EDPC_E_INVALID_ARG, "NULL argument");
    if (n_streams == 0) fail(EDPC_E_INVALID_ARG, "n_streams must be >= 1");
    if (cap < 2 * n_steps + 2) fail(EDPC_E_INVALID_ARG, "cap_per_stream < 2 * n_steps + 2");
    hipStream_t s = S(stream);
    uint64_t* d_len = nullptr;
    hip_check(hipMalloc(&d_len, n_streams * 8), "hipMalloc");
    k_rc_table_encode(d_cum, d_sym, n_steps, n_streams, d_out, cap, d_len, s);
    std::vector<uint64_t> l(n_streams);
    hipError_t e = hipMemcpyAsync(l.data(), d_len, n_streams * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_len);
    hip_check(e, "rc encode");
    for (size_t i = 0; i < n_streams; ++i) h_out_lens[i] = (uint32_t)l[i];
    return EDPC_OK;
  });
}

}  // extern "C"

// Device array behind edpc_rc_encode_noalloc: the per-stream payload
// lengths of one call (every entry below n_streams is written by the coder
// kernel before it is read back).  Each GPU holds its own copy; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) uint64_t scratch[EDPC_RC_NOALLOC_MAX_STREAMS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch array, looked up once per device.
uint64_t* scratch_ptr() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) fail(EDPC_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    g_scratch_ptr[dev] = (uint64_t*)p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

edpc_status edpc_rc_encode_noalloc(const uint32_t* d_cum, const uint8_t* d_sym, size_t n_steps,
                                   size_t n_streams, uint8_t* d_out, size_t cap,
                                   uint32_t* h_out_lens, void* stream) {
  return guarded("edpc_rc_encode_noalloc", [&] {
    if (!d_cum || !d_sym || !d_out || !h_out_lens) fail(EDPC_E_INVALID_ARG, "NULL argument");
    if (n_streams == 0) fail(EDPC_E_INVALID_ARG, "n_streams must be >= 1");
    if (n_streams > EDPC_RC_NOALLOC_MAX_STREAMS)
      fail(EDPC_E_INVALID_ARG, "n_streams exceeds EDPC_RC_NOALLOC_MAX_STREAMS");
    if (cap < 2 * n_steps + 2) fail(EDPC_E_INVALID_ARG, "cap_per_stream < 2 * n_steps + 2");
    hipStream_t s = S(stream);
    uint64_t* d_len = scratch_ptr();
    k_rc_table_encode(d_cum, d_sym, n_steps, n_streams, d_out, cap, d_len, s);
    hip_check(hipGetLastError(), "rc encode launch");
    // lengths back through a fixed host buffer, a slice at a time
    constexpr size_t kSlice = 512;
    uint64_t part[kSlice];
    for (size_t b = 0; b < n_streams; b += kSlice) {
      const size_t k = std::min(kSlice, n_streams - b);
      hip_check(hipMemcpyAsync(part, d_len + b, k * sizeof(uint64_t), hipMemcpyDeviceToHost, s),
                "copy");
      hip_check(hipStreamSynchronize(s), "rc encode");
      for (size_t i = 0; i < k; ++i) h_out_lens[b + i] = (uint32_t)part[i];
    }
    return EDPC_OK;
  });
}

edpc_status edpc_rc_decode(const uint32_t* d_cum, const uint8_t* d_in, const uint32_t* h_in_lens,
                           size_t cap, size_t n_steps, size_t n_streams, uint8_t* d_sym,
                           void* stream) {
  return guarded("edpc_rc_decode", [&] {
    if (!d_cum || !d_in || !h_in_lens || !d_sym) fail(EDPC_E_INVALID_ARG, "NULL argument");
    if (n_streams == 0) fail(EDPC_E_INVALID_ARG, "n_streams must be >= 1");
    hipStream_t s = S(stream);
    std::vector<uint64_t> l(h_in_lens, h_in_lens + n_streams);
    uint64_t* d_len = nullptr;
    hip_check(hipMalloc(&d_len, n_streams * 8), "hipMalloc");
    hipError_t e = hipMemcpyAsync(d_len, l.data(), n_streams * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      k_rc_table_decode(d_cum, d_in, d_len, cap, n_steps, n_streams, d_sym, s);
      e = hipStreamSynchronize(s);
    }
    (void)hipFree(d_len);
    hip_check(e, "rc decode");
    return EDPC_OK;
  });
}

edpc_status edpc_rc_encode_host(const uint32_t* h_cum, const uint8_t* h_sym, size_t n_steps,
                                uint8_t* h_out, size_t cap, size_t* out_len) {
  if (!h_cum || (n_steps && !h_sym) || !h_out || !out_len)
    return set_err(EDPC_E_INVALID_ARG, "NULL argument");
  if (cap < 2 * n_steps + 2) return set_err(EDPC_E_INVALID_ARG, "cap < 2 * n_steps + 2");
  RcEnc e;
  rc_enc_init(e);
  for (size_t t = 0; t < n_steps; ++t) {
    const uint32_t* c = h_cum + t * 257;
    const uint32_t x = h_sym[t];
    rc_encode(e, h_out, cap, c[x], c[x + 1] - c[x]);
  }
  rc_finish(e, h_out, cap);
  *out_len = e.pos;
  return EDPC_OK;
}

edpc_status edpc_rc_decode_host(const uint32_t* h_cum, const uint8_t* h_in, size_t in_len,
                                size_t n_steps, uint8_t* h_sym) {
  if (!h_cum || (in_len && !h_in) || (n_steps && !h_sym))
    return set_err(EDPC_E_INVALID_ARG, "NULL argument");
  RcDec d;
  rc_dec_init(d, h_in, in_len);
  for (size_t t = 0; t < n_steps; ++t) {
    const uint32_t* c = h_cum + t * 257;
    const uint32_t x = rc_find(d, c);
    rc_consume(d, h_in, in_len, c[x], c[x + 1]);
    h_sym[t] = (uint8_t)x;
  }
  return EDPC_OK;
}

}  // extern "C"
