// Host-to-host codec with the transfers overlapped with the model steps.
//
// The paper overlaps GPU prediction with CPU coding (its decoupled pipeline,
// Sec. 3.3).  Here the coder already runs on the GPU, so what remains to
// overlap is the movement of the data between host and device: the input
// (encoder) or the decoded output (decoder) passes through a device window
// of a few chunks of `chunk` steps per stream, and payload bytes that no
// later carry can change leave the device while the next chunk is coded.
//
// Encoder, chunk k (positions [k T, (k + 1) T) of every stream):
//   host     gathers the chunk of every stream into pinned staging P[k % 2]
//            (and updates the streams' CRCs), on several threads;
//   copy     one 2-D copy P[k % 2] -> window slot k % S (S T bytes per
//            stream, S = 2 + ceil(t / T)), after the steps of chunk k - 2,
//            the last ones to read that slot;
//   compute  the steps of chunk k, then the payload drain of the chunk;
//   copy     the drained bytes to pinned host memory, appended per stream by
//            the host while chunk k + 1 runs.
// The container is then assembled on the host.  The decoder mirrors it: the
// payloads go up once, the decoded chunk k leaves its window slot while
// chunk k + 1 is decoded.  Every model step is the one encoder_begin /
// decoder_begin would run, so the containers are identical.
#include <algorithm>
#include <cstring>
#include <thread>

#include "codec.h"
#include "trace.h"

namespace edpc {

namespace {

// f(i) for i in [0, n) on up to 8 host threads (one thread for small n).
template <class F>
void parallel_for(size_t n, size_t work_bytes, F&& f) {
  const size_t hw = std::max<unsigned>(1, std::thread::hardware_concurrency());
  const size_t nt = work_bytes < (1u << 20) ? 1 : std::min<size_t>({8, hw, n});
  if (nt <= 1) {
    for (size_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  for (size_t t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (size_t i = t; i < n; i += nt) f(i);
    });
  for (auto& x : th) x.join();
}

struct Pinned {
  uint8_t* p = nullptr;
  explicit Pinned(size_t bytes) {
    void* q = nullptr;
    hip_check(hipHostMalloc(&q, std::max<size_t>(bytes, 1), hipHostMallocDefault), "hipHostMalloc");
    p = (uint8_t*)q;
  }
  ~Pinned() { if (p) (void)hipHostFree(p); }
  Pinned(const Pinned&) = delete;
  Pinned& operator=(const Pinned&) = delete;
};

struct Event {
  hipEvent_t e = nullptr;
  Event() { hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate"); }
  ~Event() { if (e) (void)hipEventDestroy(e); }
  Event(const Event&) = delete;
  Event& operator=(const Event&) = delete;
};

struct CopyStream {
  hipStream_t s = nullptr;
  CopyStream() { hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate"); }
  ~CopyStream() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

void check_chunk(uint32_t chunk, uint32_t context) {
  if (chunk < context || chunk < 1 || chunk > (1u << 22))
    fail(EDPC_E_INVALID_ARG, "chunk_steps must be in [context, 2^22]");
}

// Window slots per stream: the steps of chunk k read back t bytes, so chunk
// k + 2 may overwrite what chunk k's steps read only after they finished.
uint32_t window_slots(uint32_t chunk, uint32_t context) {
  return 2 + (context + chunk - 1) / chunk;
}

// Point a session's stream table at a window of `win` bytes per stream.
void use_window(Session& ss, uint8_t* window, uint64_t win) {
  std::vector<uint64_t> off(ss.n);
  for (size_t s = 0; s < ss.n; ++s) off[s] = s * win;
  hip_check(hipMemcpyAsync(ss.d_off, off.data(), ss.n * 8, hipMemcpyHostToDevice, ss.s), "copy");
  hip_check(hipStreamSynchronize(ss.s), "copy");
  ss.io.ring = (uint32_t)win;
  ss.io.off = ss.d_off;
}

}  // namespace

size_t stream_encode(const edpc_config& cfg, const uint8_t* h_in, const uint64_t* lens, size_t n,
                     uint8_t* h_out, size_t out_cap, uint32_t chunk, hipStream_t s,
                     size_t* required) {
  Model::validate(cfg);
  if (n == 0) fail(EDPC_E_INVALID_ARG, "n_streams must be >= 1");
  if (n > EDPC_MAX_STREAMS) fail(EDPC_E_INVALID_ARG, "too many streams");
  for (size_t i = 0; i < n; ++i)
    if (lens[i] > EDPC_MAX_STREAM_LEN) fail(EDPC_E_INVALID_ARG, "stream longer than EDPC_MAX_STREAM_LEN");
  const uint32_t C = cfg.context, T = chunk;
  check_chunk(T, C);
  const uint32_t S = window_slots(T, C);
  const uint64_t W = (uint64_t)S * T;
  if (W > 0xFFFFFFFFull) fail(EDPC_E_INVALID_ARG, "chunk_steps too large for the window");

  std::unique_ptr<Session> ss(new Session());
  ss->s = s;
  ss->cfg = cfg;
  ss->n = n;
  ss->lens.assign(lens, lens + n);
  common_setup(*ss, nullptr);
  uint8_t* window = ss->dalloc<uint8_t>(n * W);
  use_window(*ss, window, W);
  std::vector<uint64_t> in_off(n), pay_off(n), pay_cap(n);
  uint64_t o = 0, po = 0;
  for (size_t i = 0; i < n; ++i) {
    in_off[i] = o;
    o += lens[i];
    pay_off[i] = po;
    pay_cap[i] = 2 * lens[i] + 8;
    po += pay_cap[i];
  }
  ss->d_pay = ss->dalloc<uint8_t>(po);
  ss->d_pay_off = ss->dalloc<uint64_t>(n);
  ss->d_pay_cap = ss->dalloc<uint64_t>(n);
  hip_check(hipMemcpyAsync(ss->d_pay_off, pay_off.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  hip_check(hipMemcpyAsync(ss->d_pay_cap, pay_cap.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  ss->d_enc = ss->dalloc<RcEnc>(n);
  ss->io.src = window;
  ss->io.pay = ss->d_pay;
  ss->io.pay_off = ss->d_pay_off;
  ss->io.pay_cap = ss->d_pay_cap;
  ss->io.enc = ss->d_enc;

  // drained payload bytes: at most 2 per step per stream plus the bytes a
  // run of 0xFF held back; the drain takes at most `stride` at a time
  const uint32_t stride = 2 * T + 64;
  uint64_t* d_done = ss->dalloc<uint64_t>(n);
  hip_check(hipMemsetAsync(d_done, 0, n * 8, s), "memset");
  uint8_t* d_drain[2] = {ss->dalloc<uint8_t>(n * (size_t)stride), ss->dalloc<uint8_t>(n * (size_t)stride)};
  uint32_t* d_dlen[2] = {ss->dalloc<uint32_t>(n), ss->dalloc<uint32_t>(n)};
  Pinned in_stage0(n * (size_t)T), in_stage1(n * (size_t)T);
  uint8_t* in_stage[2] = {in_stage0.p, in_stage1.p};
  Pinned h_drain0(n * (size_t)stride + n * 4), h_drain1(n * (size_t)stride + n * 4);
  uint8_t* h_drain[2] = {h_drain0.p, h_drain1.p};
  CopyStream cp;
  Event ev_h2d[2], ev_steps[2], ev_drained[2], ev_d2h[2];
  std::vector<std::vector<uint8_t>> pay(n);
  std::vector<uint32_t> crc(n, 0);
  std::vector<int> d2h_pending(2, 0);

  auto drain_to_host = [&](int b, bool all) {
    // the drain buffer b is free once its previous copy to the host is done
    hip_check(hipStreamWaitEvent(s, ev_d2h[b].e, 0), "wait");
    k_pay_drain(ss->d_enc, ss->d_pay, ss->d_pay_off, d_done, (int)n, all, d_drain[b], stride,
                d_dlen[b], s);
    hip_check(hipGetLastError(), "drain launch");
    hip_check(hipEventRecord(ev_drained[b].e, s), "record");
    hip_check(hipStreamWaitEvent(cp.s, ev_drained[b].e, 0), "wait");
    hip_check(hipMemcpyAsync(h_drain[b], d_drain[b], n * (size_t)stride, hipMemcpyDeviceToHost, cp.s),
              "copy");
    hip_check(hipMemcpyAsync(h_drain[b] + n * (size_t)stride, d_dlen[b], n * 4,
                             hipMemcpyDeviceToHost, cp.s), "copy");
    hip_check(hipEventRecord(ev_d2h[b].e, cp.s), "record");
    d2h_pending[b] = 1;
  };
  // append the bytes of drain buffer b to the host payloads; returns the count
  auto collect = [&](int b) -> uint64_t {
    if (!d2h_pending[b]) return 0;
    hip_check(hipEventSynchronize(ev_d2h[b].e), "sync");
    d2h_pending[b] = 0;
    const uint32_t* cnt = (const uint32_t*)(h_drain[b] + n * (size_t)stride);
    uint64_t total = 0;
    for (size_t i = 0; i < n; ++i) total += cnt[i];
    parallel_for(n, total, [&](size_t i) {
      const uint8_t* src = h_drain[b] + i * stride;
      pay[i].insert(pay[i].end(), src, src + cnt[i]);
    });
    return total;
  };

  const uint64_t maxlen = ss->maxlen;
  const uint64_t nchunks = (maxlen + T - 1) / T;
  for (uint64_t k = 0; k < nchunks; ++k) {
    TraceRange range("encode chunk");
    const int b = (int)(k & 1);
    // staging b was last copied for chunk k - 2
    if (k >= 2) hip_check(hipEventSynchronize(ev_h2d[b].e), "sync");
    const uint64_t p0 = k * T;
    uint8_t* stage = in_stage[b];
    parallel_for(n, n * (size_t)T, [&](size_t i) {
      if (lens[i] <= p0) return;
      const uint64_t cnt = std::min<uint64_t>(T, lens[i] - p0);
      std::memcpy(stage + i * (size_t)T, h_in + in_off[i] + p0, cnt);
      crc[i] = crc32_host(h_in + in_off[i] + p0, cnt, crc[i]);
    });
    // window slot k % S was last read by the steps of chunk k - 2
    if (k >= 2) hip_check(hipStreamWaitEvent(cp.s, ev_steps[b].e, 0), "wait");
    hip_check(hipMemcpy2DAsync(window + (k % S) * T, W, stage, T, T, n, hipMemcpyHostToDevice, cp.s),
              "copy");
    hip_check(hipEventRecord(ev_h2d[b].e, cp.s), "record");
    hip_check(hipStreamWaitEvent(s, ev_h2d[b].e, 0), "wait");
    if (k == 0) {
      k_uniform_prefix(ss->io, (int)n, (int)C, false, s);
      hip_check(hipGetLastError(), "prefix launch");
    }
    const uint64_t to = std::min<uint64_t>(maxlen, p0 + T);
    if (ss->next < to) ss->run(to - ss->next);
    hip_check(hipEventRecord(ev_steps[b].e, s), "record");
    drain_to_host(b, false);
    collect(b ^ 1);  // chunk k - 1's bytes, while chunk k runs
  }
  if (nchunks == 0) {  // every stream is empty
    k_uniform_prefix(ss->io, (int)n, (int)C, false, s);
  }
  // flush every coder, then drain everything that is left
  k_rc_finish(ss->io, (int)n, s);
  hip_check(hipGetLastError(), "finish launch");
  int b = (int)(nchunks & 1);
  collect(b);
  collect(b ^ 1);
  for (;;) {
    drain_to_host(b, true);
    if (collect(b) == 0) break;
    b ^= 1;
  }
  std::vector<RcEnc> enc(n);
  hip_check(hipMemcpyAsync(enc.data(), ss->d_enc, n * sizeof(RcEnc), hipMemcpyDeviceToHost, s), "copy");
  hip_check(hipStreamSynchronize(s), "encode");

  Header h;
  h.cfg = cfg;
  h.kernel_id = ss->model->kc.encode();
  h.arch = kArch;
  h.lens = ss->lens;
  h.crcs = crc;
  h.pay_lens.resize(n);
  for (size_t i = 0; i < n; ++i) {
    h.pay_lens[i] = pay[i].size();
    if (pay[i].size() != enc[i].pos || enc[i].pos > 2 * lens[i] + 2)
      fail(EDPC_E_DEVICE, "streamed payload does not match the coder state");
  }
  std::vector<uint8_t> hb = write_header(h);
  size_t total = hb.size();
  std::vector<size_t> dst(n);
  for (size_t i = 0; i < n; ++i) { dst[i] = total; total += pay[i].size(); }
  if (required) *required = total;
  if (total > out_cap) fail(EDPC_E_CAPACITY, "output buffer too small");
  std::memcpy(h_out, hb.data(), hb.size());
  parallel_for(n, total, [&](size_t i) {
    if (!pay[i].empty()) std::memcpy(h_out + dst[i], pay[i].data(), pay[i].size());
  });
  return total;
}

size_t stream_decode(const uint8_t* h_in, size_t in_len, uint8_t* h_out, size_t out_cap,
                     uint32_t chunk, hipStream_t s) {
  Header h;
  size_t need = 0;
  std::string err;
  edpc_status st = parse_header(h_in, in_len, &h, &need, &err);
  if (st != EDPC_OK) fail(st, err);
  KernelConfig kc = header_kernels(h);
  const size_t n = h.lens.size();
  if (h.total_pay > in_len || h.header_len > in_len - h.total_pay)
    fail(EDPC_E_CORRUPT, "container truncated");
  if (h.total_len > out_cap) fail(EDPC_E_CAPACITY, "output buffer too small");
  const uint32_t C = h.cfg.context, T = chunk;
  check_chunk(T, C);
  const uint32_t S = window_slots(T, C);
  const uint64_t W = (uint64_t)S * T;
  if (W > 0xFFFFFFFFull) fail(EDPC_E_INVALID_ARG, "chunk_steps too large for the window");

  std::unique_ptr<Session> ss(new Session());
  ss->decoding = true;
  ss->s = s;
  ss->cfg = h.cfg;
  ss->n = n;
  ss->lens = h.lens;
  ss->hdr = h;
  common_setup(*ss, &kc);
  uint8_t* window = ss->dalloc<uint8_t>(n * W);
  use_window(*ss, window, W);
  // the payloads go up once (they are what the decoder reads first)
  uint8_t* d_pay = ss->dalloc<uint8_t>(h.total_pay);
  if (h.total_pay)
    hip_check(hipMemcpyAsync(d_pay, h_in + h.header_len, h.total_pay, hipMemcpyHostToDevice, s), "copy");
  std::vector<uint64_t> pay_off(n), out_off(n);
  uint64_t o = 0, po = 0;
  for (size_t i = 0; i < n; ++i) {
    pay_off[i] = po;
    po += h.pay_lens[i];
    out_off[i] = o;
    o += h.lens[i];
  }
  ss->d_pay_off = ss->dalloc<uint64_t>(n);
  ss->d_pay_cap = ss->dalloc<uint64_t>(n);
  hip_check(hipMemcpyAsync(ss->d_pay_off, pay_off.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  hip_check(hipMemcpyAsync(ss->d_pay_cap, h.pay_lens.data(), n * 8, hipMemcpyHostToDevice, s), "copy");
  ss->d_dec = ss->dalloc<RcDec>(n);
  ss->io.dst = window;
  ss->io.pay_in = d_pay;
  ss->io.pay_off = ss->d_pay_off;
  ss->io.pay_cap = ss->d_pay_cap;
  ss->io.dec = ss->d_dec;
  k_uniform_prefix(ss->io, (int)n, (int)C, true, s);
  hip_check(hipGetLastError(), "prefix launch");

  Pinned out0(n * (size_t)T), out1(n * (size_t)T);
  uint8_t* out_stage[2] = {out0.p, out1.p};
  CopyStream cp;
  std::vector<Event> ev_steps(S), ev_d2h(S);
  std::vector<uint32_t> crc(n, 0);
  auto unpack = [&](uint64_t k) {
    hip_check(hipEventSynchronize(ev_d2h[k % S].e), "sync");
    const uint64_t p0 = k * T;
    const uint8_t* stage = out_stage[k & 1];
    parallel_for(n, n * (size_t)T, [&](size_t i) {
      if (h.lens[i] <= p0) return;
      const uint64_t cnt = std::min<uint64_t>(T, h.lens[i] - p0);
      std::memcpy(h_out + out_off[i] + p0, stage + i * (size_t)T, cnt);
      crc[i] = crc32_host(stage + i * (size_t)T, cnt, crc[i]);
    });
  };
  const uint64_t maxlen = ss->maxlen;
  const uint64_t nchunks = (maxlen + T - 1) / T;
  for (uint64_t k = 0; k < nchunks; ++k) {
    TraceRange range("decode chunk");
    const uint32_t slot = (uint32_t)(k % S);
    // the slot's previous chunk (k - S) must have left for the host
    if (k >= S) hip_check(hipStreamWaitEvent(s, ev_d2h[slot].e, 0), "wait");
    const uint64_t to = std::min<uint64_t>(maxlen, (k + 1) * T);
    if (ss->next < to) ss->run(to - ss->next);
    hip_check(hipEventRecord(ev_steps[slot].e, s), "record");
    // staging k & 1 held chunk k - 2, unpacked at iteration k - 1
    hip_check(hipStreamWaitEvent(cp.s, ev_steps[slot].e, 0), "wait");
    hip_check(hipMemcpy2DAsync(out_stage[k & 1], T, window + (uint64_t)slot * T, W, T, n,
                               hipMemcpyDeviceToHost, cp.s), "copy");
    hip_check(hipEventRecord(ev_d2h[slot].e, cp.s), "record");
    if (k >= 1) unpack(k - 1);  // while chunk k runs
  }
  if (nchunks) unpack(nchunks - 1);
  hip_check(hipStreamSynchronize(s), "decode");
  size_t total = 0;
  for (size_t i = 0; i < n; ++i) {
    total += h.lens[i];
    if (crc[i] != h.crcs[i]) fail(EDPC_E_CHECKSUM, "decoded data CRC mismatch");
  }
  return total;
}

}  // namespace edpc
