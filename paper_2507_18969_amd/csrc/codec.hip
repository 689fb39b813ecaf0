// Multi-stream codec sessions and the container.
#include "codec.h"
#include "trace.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>

namespace edpc {

uint32_t crc32_host(const uint8_t* p, size_t n, uint32_t c) {
  static uint32_t table[256];
  static bool init = false;
  if (!init) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t v = i;
      for (int k = 0; k < 8; ++k) v = (v & 1u) ? (0xEDB88320u ^ (v >> 1)) : (v >> 1);
      table[i] = v;
    }
    init = true;
  }
  c = ~c;
  for (size_t i = 0; i < n; ++i) c = table[(c ^ p[i]) & 0xFFu] ^ (c >> 8);
  return ~c;
}

namespace {
struct Writer {
  std::vector<uint8_t> b;
  void u16(uint16_t v) { for (int i = 0; i < 2; ++i) b.push_back((uint8_t)(v >> (8 * i))); }
  void u32(uint32_t v) { for (int i = 0; i < 4; ++i) b.push_back((uint8_t)(v >> (8 * i))); }
  void u64(uint64_t v) { for (int i = 0; i < 8; ++i) b.push_back((uint8_t)(v >> (8 * i))); }
  void f32(float f) { uint32_t u; std::memcpy(&u, &f, 4); u32(u); }
};
uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
uint32_t rd32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
uint64_t rd64(const uint8_t* p) { return (uint64_t)rd32(p) | ((uint64_t)rd32(p + 4) << 32); }
float rdf(const uint8_t* p) { uint32_t u = rd32(p); float f; std::memcpy(&f, &u, 4); return f; }
}  // namespace

std::vector<uint8_t> write_header(const Header& h) {
  Writer w;
  w.b.insert(w.b.end(), {'E', 'D', 'P', 'C'});
  w.u16(kFormatVersion);
  w.u16(0);
  const size_t n = h.lens.size();
  w.u32((uint32_t)(kHeaderFixed + kPerStream * n + 4));
  w.u32((uint32_t)n);
  const edpc_config& c = h.cfg;
  for (uint32_t v : {c.context, c.embed, c.latent, c.blocks, c.hidden, c.branches, c.cdf_bits,
                     c.precision, c.flags})
    w.u32(v);
  for (float f : {c.lr, c.beta1, c.beta2, c.eps}) w.f32(f);
  w.u64(c.seed);
  w.u64(h.kernel_id);
  w.u32(h.arch);
  w.u32(0);
  for (size_t s = 0; s < n; ++s) {
    w.u64(h.lens[s]);
    w.u64(h.pay_lens[s]);
    w.u32(h.crcs[s]);
  }
  w.u32(crc32_host(w.b.data(), w.b.size()));
  return w.b;
}

edpc_status parse_header(const uint8_t* p, size_t len, Header* h, size_t* need, std::string* err) {
  *need = kHeaderFixed + 4;
  if (len < 16) { *err = "container shorter than its fixed header"; return EDPC_E_CORRUPT; }
  if (std::memcmp(p, "EDPC", 4) != 0) { *err = "bad magic"; return EDPC_E_CORRUPT; }
  if (rd16(p + 4) != kFormatVersion) { *err = "unsupported format version"; return EDPC_E_UNSUPPORTED; }
  const uint32_t hl = rd32(p + 8), n = rd32(p + 12);
  if (n == 0 || n > EDPC_MAX_STREAMS) { *err = "stream count out of range"; return EDPC_E_CORRUPT; }
  if ((uint64_t)hl != kHeaderFixed + (uint64_t)kPerStream * n + 4) {
    *err = "inconsistent header length";
    return EDPC_E_CORRUPT;
  }
  *need = hl;
  if (len < hl) { *err = "container shorter than its header"; return EDPC_E_CORRUPT; }
  if (crc32_host(p, hl - 4) != rd32(p + hl - 4)) { *err = "header CRC mismatch"; return EDPC_E_CHECKSUM; }
  edpc_config& c = h->cfg;
  std::memset(&c, 0, sizeof(c));
  c.struct_size = sizeof(edpc_config);
  uint32_t* f[] = {&c.context, &c.embed, &c.latent, &c.blocks, &c.hidden, &c.branches, &c.cdf_bits,
                   &c.precision, &c.flags};
  for (int i = 0; i < 9; ++i) *f[i] = rd32(p + 16 + 4 * i);
  c.lr = rdf(p + 52);
  c.beta1 = rdf(p + 56);
  c.beta2 = rdf(p + 60);
  c.eps = rdf(p + 64);
  c.seed = rd64(p + 68);
  h->kernel_id = rd64(p + 76);
  h->arch = rd32(p + 84);
  h->lens.resize(n);
  h->pay_lens.resize(n);
  h->crcs.resize(n);
  // Each length is bounded before any arithmetic on it (2 len + 2 cannot
  // wrap), and the totals are summed with overflow checks, so that no later
  // offset computed from the header can leave the caller's buffers.
  uint64_t total = 0, pay_total = 0;
  for (uint32_t s = 0; s < n; ++s) {
    const uint8_t* q = p + kHeaderFixed + kPerStream * s;
    h->lens[s] = rd64(q);
    h->pay_lens[s] = rd64(q + 8);
    h->crcs[s] = rd32(q + 16);
    if (h->lens[s] > EDPC_MAX_STREAM_LEN) {
      *err = "stream length out of range";
      return EDPC_E_CORRUPT;
    }
    if (h->pay_lens[s] > 2 * h->lens[s] + 2 || (h->lens[s] == 0) != (h->pay_lens[s] == 0)) {
      *err = "payload length out of range";
      return EDPC_E_CORRUPT;
    }
    if (__builtin_add_overflow(total, h->lens[s], &total) ||
        __builtin_add_overflow(pay_total, h->pay_lens[s], &pay_total)) {
      *err = "stream lengths overflow";
      return EDPC_E_CORRUPT;
    }
  }
  h->total_len = total;
  h->total_pay = pay_total;
  h->header_len = hl;
  return EDPC_OK;
}

size_t encode_bound(const edpc_config& cfg, const uint64_t* lens, size_t n) {
  (void)cfg;
  if (n > EDPC_MAX_STREAMS) fail(EDPC_E_INVALID_ARG, "too many streams");
  size_t b = kHeaderFixed + kPerStream * n + 4;
  for (size_t s = 0; s < n; ++s) {
    if (lens[s] > EDPC_MAX_STREAM_LEN) fail(EDPC_E_INVALID_ARG, "stream longer than EDPC_MAX_STREAM_LEN");
    b += 2 * lens[s] + 2;
  }
  return b;
}

Session::~Session() {
  if (s) (void)hipStreamSynchronize(s);
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  if (cap) (void)hipStreamDestroy(cap);
  model.reset();
  for (void* p : allocs) (void)hipFree(p);
}

template <class T>
T* Session::dalloc(size_t cnt) {
  void* p = nullptr;
  if (cnt == 0) cnt = 1;
  hip_check(hipMalloc(&p, cnt * sizeof(T)), "hipMalloc");
  allocs.push_back(p);
  return (T*)p;
}

int Session::rows_at(uint64_t i) const {
  // number of streams longer than i (lens_sorted is decreasing)
  auto it = std::partition_point(lens_sorted.begin(), lens_sorted.end(),
                                 [&](int64_t l) { return (uint64_t)l > i; });
  return (int)(it - lens_sorted.begin());
}

int Session::bucket(int rows) const {
  // grid rows of a captured window: rows rounded up to a multiple of 128
  const int b = ((rows + 127) / 128) * 128;
  return std::min(b, (int)model->max_rows);
}

void Session::step_direct(uint64_t i, int grid_rows, bool explicit_step, hipStream_t st, int rel) {
  KTimer* timer = model->timer;
  StepOutputs out;
  out.update = true;
  if (model->kc.fused) {
    // the row-block step's first kernel forms the step state
    const StepSched sc{sched, explicit_step ? 1 : 2, explicit_step ? (int)i : rel};
    model->step(decoding ? MODE_DECODE : MODE_ENCODE, io, out, grid_rows, st, &sc);
    return;
  }
  if (timer) timer->begin(KC_SCHEDULE, st);
  k_step_schedule(model->st, sched, explicit_step ? (int)i : -1, st);
  if (timer) timer->end(st);
  if (timer) timer->begin(KC_GATHER, st);
  k_gather(model->st, io, model->C, model->ctx, model->tgt, grid_rows, decoding, st);
  if (timer) timer->end(st);
  model->step(decoding ? MODE_DECODE : MODE_ENCODE, io, out, grid_rows, st);
}

// Steps next .. next+k-1.  Windows of graph_steps steps whose active rows fall
// in one bucket replay a captured graph (each kernel reads the step number and
// row count from the device-side step state); the rest launch directly.  The
// graphs are captured on a private stream and launched on the session's.
void Session::run(uint64_t k) {
  const uint64_t end = std::min(maxlen, next + k);
  uint64_t i = next;
  const bool use_graphs = graph_steps > 0 && model->timer == nullptr;
  while (i < end) {
    const int rows = rows_at(i);
    if (use_graphs && i + graph_steps <= end) {
      const int b = bucket(rows);
      if (bucket(rows_at(i + graph_steps - 1)) == b) {
        auto it = graphs.find(b);
        if (it == graphs.end()) {
          if (!cap) hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "stream");
          TraceRange range("graph capture");
          hipGraph_t g = nullptr;
          hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "capture");
          try {
            for (int q = 0; q < graph_steps; ++q) step_direct(0, b, false, cap, q + 1);
          } catch (...) {
            (void)hipStreamEndCapture(cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          hip_check(hipStreamEndCapture(cap, &g), "capture");
          hipGraphExec_t ex;
          const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          hip_check(e, "graph instantiate");
          it = graphs.emplace(b, ex).first;
        }
        // the captured steps advance from the device step counter
        TraceRange range("graph window");
        k_step_set(model->st, (int)i - 1, s);
        hip_check(hipGraphLaunch(it->second, s), "graph launch");
        i += graph_steps;
        continue;
      }
    }
    {
      TraceRange range("direct step");
      step_direct(i, rows, true, s);
    }
    ++i;
  }
  next = end;
}

void common_setup(Session& ss, const KernelConfig* kc) {
  const size_t n = ss.n;
  std::vector<uint32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0u);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](uint32_t a, uint32_t b) { return ss.lens[a] > ss.lens[b]; });
  ss.perm = perm;
  ss.lens_sorted.resize(n);
  for (size_t r = 0; r < n; ++r) ss.lens_sorted[r] = (int64_t)ss.lens[perm[r]];
  ss.maxlen = n ? (uint64_t)ss.lens_sorted[0] : 0;
  const size_t rows = std::max<size_t>(1, (size_t)ss.rows_at(ss.cfg.context));
  ss.model.reset(new Model(ss.cfg, n, rows, kc));
  ss.model->init_params(ss.s);
  ss.model->build_tables(ss.s);
  if (!ss.decoding && (ss.cfg.flags & EDPC_CFG_AUTOTUNE)) {
    TraceRange range("autotune");
    ss.model->autotune(ss.s);
  }
  hip_check(hipMemcpyAsync(ss.model->slot, perm.data(), std::min(n, rows) * sizeof(uint32_t),
                           hipMemcpyHostToDevice, ss.s), "copy");
  ss.d_lens_sorted = ss.dalloc<int64_t>(n);
  hip_check(hipMemcpyAsync(ss.d_lens_sorted, ss.lens_sorted.data(), n * sizeof(int64_t),
                           hipMemcpyHostToDevice, ss.s), "copy");
  ss.d_lens = ss.dalloc<uint64_t>(n);
  hip_check(hipMemcpyAsync(ss.d_lens, ss.lens.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice,
                           ss.s), "copy");
  std::vector<uint64_t> off(n);
  uint64_t o = 0;
  for (size_t s = 0; s < n; ++s) { off[s] = o; o += ss.lens[s]; }
  ss.d_off = ss.dalloc<uint64_t>(n);
  hip_check(hipMemcpyAsync(ss.d_off, off.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice, ss.s),
            "copy");
  ss.d_crc = ss.dalloc<uint32_t>(n);
  ss.sched.lens_sorted = ss.d_lens_sorted;
  ss.sched.n = (int)n;
  ss.sched.context = (int)ss.cfg.context;
  ss.sched.beta1 = ss.cfg.beta1;
  ss.sched.beta2 = ss.cfg.beta2;
  std::memset(&ss.io, 0, sizeof(ss.io));
  ss.io.slot = ss.model->slot;
  ss.io.off = ss.d_off;
  ss.io.lens = ss.d_lens;
  ss.next = std::min<uint64_t>(ss.cfg.context, ss.maxlen);
  ss.graph_steps = (ss.cfg.flags & EDPC_CFG_NO_GRAPHS) ? 0 : kGraphSteps;
}

std::unique_ptr<Session> encoder_begin(const edpc_config& cfg, const uint8_t* d_in,
                                       const uint64_t* lens, size_t n, hipStream_t s,
                                       const KernelConfig* kc) {
  Model::validate(cfg);
  if (n == 0) fail(EDPC_E_INVALID_ARG, "n_streams must be >= 1");
  if (n > EDPC_MAX_STREAMS) fail(EDPC_E_INVALID_ARG, "too many streams");
  for (size_t i = 0; i < n; ++i)
    if (lens[i] > EDPC_MAX_STREAM_LEN) fail(EDPC_E_INVALID_ARG, "stream longer than EDPC_MAX_STREAM_LEN");
  std::unique_ptr<Session> ss(new Session());
  ss->s = s;
  ss->cfg = cfg;
  ss->n = n;
  ss->lens.assign(lens, lens + n);
  common_setup(*ss, kc);
  std::vector<uint64_t> pay_off(n), pay_cap(n);
  uint64_t o = 0;
  for (size_t i = 0; i < n; ++i) { pay_off[i] = o; pay_cap[i] = 2 * lens[i] + 8; o += pay_cap[i]; }
  ss->d_pay = ss->dalloc<uint8_t>(o);
  ss->d_pay_off = ss->dalloc<uint64_t>(n);
  ss->d_pay_cap = ss->dalloc<uint64_t>(n);
  hip_check(hipMemcpyAsync(ss->d_pay_off, pay_off.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  hip_check(hipMemcpyAsync(ss->d_pay_cap, pay_cap.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  ss->d_enc = ss->dalloc<RcEnc>(n);
  ss->io.src = d_in;
  ss->io.pay = ss->d_pay;
  ss->io.pay_off = ss->d_pay_off;
  ss->io.pay_cap = ss->d_pay_cap;
  ss->io.enc = ss->d_enc;
  k_crc32(d_in, ss->d_off, ss->d_lens, (int)n, ss->d_crc, s);
  k_uniform_prefix(ss->io, (int)n, (int)cfg.context, false, s);
  hip_check(hipGetLastError(), "encoder setup");
  return ss;
}

size_t encoder_finish(Session& ss, uint8_t* d_out, size_t out_cap) {
  ss.run(ss.maxlen);
  TraceRange range("container");
  k_rc_finish(ss.io, (int)ss.n, ss.s);
  std::vector<RcEnc> enc(ss.n);
  Header h;
  h.cfg = ss.cfg;
  h.kernel_id = ss.model->kc.encode();
  h.arch = kArch;
  h.lens = ss.lens;
  h.crcs.resize(ss.n);
  hip_check(hipMemcpyAsync(enc.data(), ss.d_enc, ss.n * sizeof(RcEnc), hipMemcpyDeviceToHost, ss.s),
            "copy");
  hip_check(hipMemcpyAsync(h.crcs.data(), ss.d_crc, ss.n * 4, hipMemcpyDeviceToHost, ss.s), "copy");
  hip_check(hipStreamSynchronize(ss.s), "encode");
  h.pay_lens.resize(ss.n);
  for (size_t i = 0; i < ss.n; ++i) {
    h.pay_lens[i] = enc[i].pos;
    if (enc[i].pos > 2 * ss.lens[i] + 2) fail(EDPC_E_DEVICE, "payload exceeded its bound");
  }
  std::vector<uint8_t> hb = write_header(h);
  size_t total = hb.size();
  std::vector<uint64_t> dst_off(ss.n);
  for (size_t i = 0; i < ss.n; ++i) { dst_off[i] = total; total += h.pay_lens[i]; }
  if (total > out_cap) {
    Error e{EDPC_E_CAPACITY, "output buffer too small"};
    ss.out_cap = total;
    throw e;
  }
  uint64_t* d_dst_off = ss.dalloc<uint64_t>(ss.n);
  uint64_t* d_pl = ss.dalloc<uint64_t>(ss.n);
  hip_check(hipMemcpyAsync(d_dst_off, dst_off.data(), ss.n * 8, hipMemcpyHostToDevice, ss.s), "copy");
  hip_check(hipMemcpyAsync(d_pl, h.pay_lens.data(), ss.n * 8, hipMemcpyHostToDevice, ss.s), "copy");
  hip_check(hipMemcpyAsync(d_out, hb.data(), hb.size(), hipMemcpyHostToDevice, ss.s), "copy");
  k_gather_payloads(ss.d_pay, ss.d_pay_off, d_pl, d_dst_off, d_out, (int)ss.n, ss.s);
  hip_check(hipStreamSynchronize(ss.s), "encode finish");
  return total;
}

KernelConfig header_kernels(const Header& h) {
  if (h.arch != kArch) fail(EDPC_E_UNSUPPORTED, "container written for another device architecture");
  KernelConfig kc;
  if (!KernelConfig::decode(h.kernel_id, &kc)) fail(EDPC_E_UNSUPPORTED, "unknown kernel configuration");
  Model::validate(h.cfg);
  return kc;
}

std::unique_ptr<Session> decoder_begin(const uint8_t* d_in, size_t in_len, uint8_t* d_out,
                                       size_t out_cap, hipStream_t s) {
  std::vector<uint8_t> fixed(std::min<size_t>(in_len, 16));
  if (in_len < 16) fail(EDPC_E_CORRUPT, "container shorter than its fixed header");
  hip_check(hipMemcpyAsync(fixed.data(), d_in, 16, hipMemcpyDeviceToHost, s), "copy");
  hip_check(hipStreamSynchronize(s), "copy");
  Header h;
  size_t need = 0;
  std::string err;
  edpc_status st = parse_header(fixed.data(), 16, &h, &need, &err);
  if (st != EDPC_OK && err != "container shorter than its header") fail(st, err);
  if (need > in_len) fail(EDPC_E_CORRUPT, "container shorter than its header");
  std::vector<uint8_t> hb(need);
  hip_check(hipMemcpyAsync(hb.data(), d_in, need, hipMemcpyDeviceToHost, s), "copy");
  hip_check(hipStreamSynchronize(s), "copy");
  st = parse_header(hb.data(), hb.size(), &h, &need, &err);
  if (st != EDPC_OK) fail(st, err);
  KernelConfig kc = header_kernels(h);
  const size_t n = h.lens.size();
  // (parse_header bounded every length and checked both sums)
  if (h.total_pay > in_len || h.header_len > in_len - h.total_pay)
    fail(EDPC_E_CORRUPT, "container truncated");
  if (h.total_len > out_cap) fail(EDPC_E_CAPACITY, "output buffer too small");
  std::unique_ptr<Session> ss(new Session());
  ss->decoding = true;
  ss->s = s;
  ss->cfg = h.cfg;
  ss->n = n;
  ss->lens = h.lens;
  ss->hdr = h;
  ss->d_dst = d_out;
  ss->out_cap = out_cap;
  common_setup(*ss, &kc);
  std::vector<uint64_t> pay_off(n);
  uint64_t o = h.header_len;
  for (size_t i = 0; i < n; ++i) { pay_off[i] = o; o += h.pay_lens[i]; }
  ss->d_pay_off = ss->dalloc<uint64_t>(n);
  ss->d_pay_cap = ss->dalloc<uint64_t>(n);
  hip_check(hipMemcpyAsync(ss->d_pay_off, pay_off.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  hip_check(hipMemcpyAsync(ss->d_pay_cap, h.pay_lens.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  ss->d_dec = ss->dalloc<RcDec>(n);
  ss->io.dst = d_out;
  ss->io.pay_in = d_in;
  ss->io.pay_off = ss->d_pay_off;
  ss->io.pay_cap = ss->d_pay_cap;
  ss->io.dec = ss->d_dec;
  k_uniform_prefix(ss->io, (int)n, (int)h.cfg.context, true, s);
  hip_check(hipGetLastError(), "decoder setup");
  return ss;
}

size_t decoder_finish(Session& ss) {
  ss.run(ss.maxlen);
  k_crc32(ss.d_dst, ss.d_off, ss.d_lens, (int)ss.n, ss.d_crc, ss.s);
  std::vector<uint32_t> crc(ss.n);
  hip_check(hipMemcpyAsync(crc.data(), ss.d_crc, ss.n * 4, hipMemcpyDeviceToHost, ss.s), "copy");
  hip_check(hipStreamSynchronize(ss.s), "decode");
  size_t total = 0;
  for (size_t i = 0; i < ss.n; ++i) {
    total += ss.lens[i];
    if (crc[i] != ss.hdr.crcs[i]) fail(EDPC_E_CHECKSUM, "decoded data CRC mismatch");
  }
  return total;
}

}  // namespace edpc
