// Multi-stream codec sessions (Algorithm 1 over b streams in lockstep) and
// the container format.
#pragma once
#include <map>
#include <memory>
#include <vector>

#include "model.h"

namespace edpc {

// Container layout (little-endian):
//   0   "EDPC"                      magic
//   4   u16 format version (1)
//   6   u16 reserved (0)
//   8   u32 header length           96 + 20 * n_streams
//   12  u32 n_streams
//   16  u32 context, embed, latent, blocks, hidden, branches, cdf_bits,
//           precision, flags
//   52  f32 lr, beta1, beta2, eps
//   68  u64 seed
//   76  u64 kernel configuration id: 4 bits of tile choice per product slot,
//           bit 47 the BF16 row-block fused step, bit 46 the LayerNorm adjoint
//           with its column sums (layer-by-layer step), bits 48.. the numerics
//           revision
//   84  u32 device architecture (950 for gfx950)
//   88  u32 reserved (0)
//   92  per stream: u64 length, u64 payload length, u32 CRC-32 of the bytes
//   ... u32 CRC-32 of every header byte before it
//   payloads, stream order
constexpr uint16_t kFormatVersion = 1;
constexpr uint32_t kArch = 950;
constexpr size_t kHeaderFixed = 92;
constexpr size_t kPerStream = 20;
constexpr int kGraphSteps = 32;  // steps per captured window of a session

struct Header {
  edpc_config cfg;
  uint64_t kernel_id;
  uint32_t arch;
  std::vector<uint64_t> lens, pay_lens;
  std::vector<uint32_t> crcs;
  uint64_t total_len = 0, total_pay = 0;  // sums of lens / pay_lens (checked)
  size_t header_len;
};

uint32_t crc32_host(const uint8_t* p, size_t n, uint32_t c = 0);
std::vector<uint8_t> write_header(const Header& h);
// Parses and validates; returns the status and fills `h` (lengths may be
// partial when the buffer is short: then *need is the header length).
edpc_status parse_header(const uint8_t* buf, size_t len, Header* h, size_t* need, std::string* err);

struct Session {
  bool decoding = false;
  hipStream_t s = nullptr;
  edpc_config cfg;
  size_t n = 0;
  std::vector<uint64_t> lens;
  std::vector<int64_t> lens_sorted;
  std::vector<uint32_t> perm;
  uint64_t maxlen = 0, next = 0;
  std::unique_ptr<Model> model;
  std::vector<void*> allocs;
  uint64_t *d_off = nullptr, *d_lens = nullptr, *d_pay_off = nullptr, *d_pay_cap = nullptr;
  int64_t* d_lens_sorted = nullptr;
  uint32_t* d_crc = nullptr;
  RcEnc* d_enc = nullptr;
  RcDec* d_dec = nullptr;
  uint8_t* d_pay = nullptr;
  uint8_t* d_dst = nullptr;
  size_t out_cap = 0;
  Header hdr;  // decoder
  StreamIO io;
  Schedule sched;

  // captured step windows: grid-row bucket -> executable graph of graph_steps steps
  int graph_steps = 0;
  std::map<int, hipGraphExec_t> graphs;
  hipStream_t cap = nullptr;  // private non-blocking stream used only for capture

  ~Session();
  int rows_at(uint64_t i) const;
  int bucket(int rows) const;
  void run(uint64_t k);
  // explicit_step: step i; else step st->base + rel (rel-th step of a window)
  void step_direct(uint64_t i, int grid_rows, bool explicit_step, hipStream_t st, int rel = 1);
  template <class T>
  T* dalloc(size_t n);
};

std::unique_ptr<Session> encoder_begin(const edpc_config& cfg, const uint8_t* d_in,
                                       const uint64_t* lens, size_t n, hipStream_t s,
                                       const KernelConfig* kc);
size_t encoder_finish(Session& ss, uint8_t* d_out, size_t out_cap);
std::unique_ptr<Session> decoder_begin(const uint8_t* d_in, size_t in_len, uint8_t* d_out,
                                       size_t out_cap, hipStream_t s);
size_t decoder_finish(Session& ss);
size_t encode_bound(const edpc_config& cfg, const uint64_t* lens, size_t n);
// Sorting, model, schedule and stream tables of a session (cfg, n, lens, s
// and decoding already set).
void common_setup(Session& ss, const KernelConfig* kc);
// Checks a parsed header against the library (architecture, kernel
// configuration, model) and returns its kernel configuration.
KernelConfig header_kernels(const Header& h);

// Host-to-host codec (stream.hip): the same containers as encoder_begin /
// decoder_begin + finish, with the input (or the decoded output) moving
// through a device window of a few chunks of `chunk` steps per stream, the
// copies on a second stream overlapped with the steps.
size_t stream_encode(const edpc_config& cfg, const uint8_t* h_in, const uint64_t* lens, size_t n,
                     uint8_t* h_out, size_t out_cap, uint32_t chunk, hipStream_t s,
                     size_t* required);
size_t stream_decode(const uint8_t* h_in, size_t in_len, uint8_t* h_out, size_t out_cap,
                     uint32_t chunk, hipStream_t s);

}  // namespace edpc
