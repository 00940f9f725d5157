// Host runtime and C ABI: model upload, contexts, and the encode / decode /
// level_probs pipelines.  Every stage is one launch per depth (or per layer
// position) over the rows of all frames of a call, driven by segment and
// tile tables that are uploaded once per phase.
#include <array>
#include <map>
#include <mutex>

#include <algorithm>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>

#include "lpcc_internal.h"

using namespace lpcc;

// ===========================================================================
// Model
// ===========================================================================
struct HostLayer {
  int kind, depth, j, taps, cin, cout;
  int32_t m_pos, m_neg, r, z_in, z_out;
  std::vector<int32_t> bias;
  std::vector<int8_t> W;  // [taps][cin][cout] (a copy of the owner's when shared)
  int owner = 0;          // index of the layer whose weights these are (itself unless shared)
};

struct lpcc_model {
  int device = 0;
  int C = 0, D = 0, n_deep = 0, k0 = 0;
  int xfp = 1;                   // 0: the ablation schedule without cross-scale propagation
  uint32_t blob_id = 0;
  std::vector<int> first;        // first layer index of each depth (size D+1)
  std::vector<HostLayer> host;   // parsed layers
  LayerDev* d_layers = nullptr;  // device copies of the descriptors
  std::vector<LayerDev> h_layers;  // the same descriptors on the host (kernel arguments)
  void* d_mem = nullptr;         // packed weights, biases, corrections, table
  int32_t* d_lut = nullptr;
};

namespace {

uint32_t rd32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

uint32_t fnv1a(const uint8_t* p, size_t n) {
  uint32_t h = 2166136261u;
  for (size_t i = 0; i < n; i++) {
    h ^= p[i];
    h *= 16777619u;
  }
  return h;
}

// layer sequence of coded depth d: (kind, j, taps, cin, cout)
struct Spec {
  int kind, j, taps, cin, cout;
};
// Without cross-scale propagation (xfp = 0) a shallow depth starts with an
// embedding of the parent codes, and the deep ResBlock reads G alone (C -> C,
// identity skip, no skip layer).
std::vector<Spec> depth_layers(int C, int D, int n_deep, int xfp, int d) {
  const int k0 = D - n_deep - 1;
  std::vector<Spec> v;
  if (d >= 1 && d <= k0) {
    if (!xfp) v.push_back({K_EMB, d - 1, 1, 8, C});
    v.push_back({K_CONV1, 0, 27, C, C});
    v.push_back({K_CONV2, 0, 27, C, C});
    v.push_back({K_UP, d - 1, 1, C + 8, 8 * C});
  } else if (d > k0) {
    v.push_back({K_EMB, d - 1, 1, 8, C});
    for (int j = d - 1; j > k0; j--) v.push_back({K_DOWN, j, 8, C, C});
    v.push_back({K_CONV1, k0, 27, xfp ? 2 * C : C, C});
    v.push_back({K_CONV2, k0, 27, C, C});
    if (xfp) v.push_back({K_SKIP, k0, 1, 2 * C, C});
    for (int j = k0; j < d; j++) v.push_back({K_UP, j, 1, C + 8, 8 * C});
  }
  v.push_back({K_FC1, d, 1, C, C});
  v.push_back({K_FC2, d, 1, C, kNSym});
  return v;
}

// Exponent table of the integer softmax, E[i] = round(2^15 e^{-i/16}), built
// with integers only: T_0 = 2^31, T_{i+1} = round(T_i * round(2^32 e^{-1/16}) / 2^32),
// E[i] = round(T_i / 2^16).  (Equal to the rounded exponential for all i.)
void softmax_table(int32_t* E) {
  uint64_t T = 1ull << 31;
  for (int i = 0; i < 256; i++) {
    E[i] = (int32_t)((T + (1ull << 15)) >> 16);
    T = (T * 4034748382ull + (1ull << 31)) >> 32;
  }
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int parse_blob(const uint8_t* b, size_t len, lpcc_model* m) {
  if (len < 32 || rd32(b) != 0x5743504Cu) return LPCC_E_MODEL;
  const uint32_t ver = rd32(b + 4);
  if ((ver & 0xFFu) != 1 && (ver & 0xFFu) != 2) return LPCC_E_MODEL;
  if (ver & ~0x1FFu) return LPCC_E_MODEL;
  const bool shared = (ver & 0x100u) != 0;  // level-aware parameter sharing: owner index per record
  m->xfp = (ver & 0xFFu) == 1;
  m->C = (int)rd32(b + 8);
  m->D = (int)rd32(b + 12);
  m->n_deep = (int)rd32(b + 16);
  const int n_layers = (int)rd32(b + 20);
  if (!(m->C == 16 || m->C == 32 || m->C == 64)) return LPCC_E_MODEL;  // widths with kernels
  if (m->D < 1 || m->D > kMaxD || m->n_deep < 0 || m->n_deep > m->D - 1) return LPCC_E_MODEL;
  m->k0 = m->D - m->n_deep - 1;
  m->blob_id = fnv1a(b, len);
  size_t off = 32;
  m->first.assign(m->D + 1, 0);
  for (int d = 0; d < m->D; d++) {
    m->first[d] = (int)m->host.size();
    for (const Spec& sp : depth_layers(m->C, m->D, m->n_deep, m->xfp, d)) {
      if (off + 44 > len) return LPCC_E_MODEL;
      HostLayer L;
      L.kind = (int)rd32(b + off);
      L.depth = (int)rd32(b + off + 4);
      L.j = (int)rd32(b + off + 8);
      L.taps = (int)rd32(b + off + 12);
      L.cin = (int)rd32(b + off + 16);
      L.cout = (int)rd32(b + off + 20);
      L.m_pos = (int32_t)rd32(b + off + 24);
      L.m_neg = (int32_t)rd32(b + off + 28);
      L.r = (int32_t)rd32(b + off + 32);
      L.z_in = (int32_t)rd32(b + off + 36);
      L.z_out = (int32_t)rd32(b + off + 40);
      if (L.kind != sp.kind || L.depth != d || L.j != sp.j || L.taps != sp.taps || L.cin != sp.cin ||
          L.cout != sp.cout)
        return LPCC_E_MODEL;
      if (L.m_pos < 0 || L.m_neg < 0 || L.r < 0 || L.r > 62 || L.z_in < -128 || L.z_in > 127 || L.z_out < -128 ||
          L.z_out > 127)
        return LPCC_E_MODEL;
      off += 44;
      const int idx = (int)m->host.size();
      L.owner = idx;
      if (shared) {
        if (off + 4 > len) return LPCC_E_MODEL;
        L.owner = (int)rd32(b + off);
        off += 4;
        if (L.owner < 0 || L.owner > idx) return LPCC_E_MODEL;
        if (L.owner < idx) {
          const HostLayer& O = m->host[L.owner];
          if (O.owner != L.owner || O.taps != L.taps || O.cin != L.cin || O.cout != L.cout) return LPCC_E_MODEL;
        }
      }
      const size_t nb = (size_t)L.cout * 4, nw = L.owner == idx ? (size_t)L.taps * L.cin * L.cout : 0;
      if (off + nb + nw > len) return LPCC_E_MODEL;
      L.bias.resize(L.cout);
      for (int o = 0; o < L.cout; o++) {
        L.bias[o] = (int32_t)rd32(b + off + 4 * (size_t)o);
        if (L.bias[o] <= -(1 << 24) || L.bias[o] >= (1 << 24)) return LPCC_E_MODEL;
      }
      off += nb;
      if (L.owner == idx) L.W.assign((const int8_t*)(b + off), (const int8_t*)(b + off + nw));
      else L.W = m->host[L.owner].W;
      off = align_up(off + nw, 4);
      m->host.push_back(std::move(L));
    }
  }
  m->first[m->D] = (int)m->host.size();
  if ((int)m->host.size() != n_layers || off != len) return LPCC_E_MODEL;
  return LPCC_OK;
}

// Device image of one layer: packed B operand, bias (zero point folded in for
// dense layers), per-tap zero-point corrections for sparse layers.
// Requantisation q(a) = ((a m + 2^(r-1)) >> r) + z_out with m = m_pos for
// a >= 0, m_neg below (m >= 0, so q is non-decreasing on each side of 0),
// then clamped to int8.  The kernels clamp the accumulator to [a_lo, a_hi]
// first: a_hi is the smallest a >= 0 with q(a) >= 127 (int32 max if none),
// a_lo the largest a < 0 with q(a) <= -128 (int32 min if none), so every
// output is unchanged.  Inside the range |q| < 2^30 + 2^8 when r >= 1; with
// r = 0 a multiplier above 256 already saturates every nonzero accumulator,
// so it is lowered to 256, which keeps the function and the bound.
struct RqBounds {
  int32_t m_pos, m_neg, a_lo, a_hi;
};

int64_t requant_q(int64_t a, int64_t m, int r, int z) {
  const int64_t rnd = r > 0 ? (1ll << (r - 1)) : 0;
  return ((a * m + rnd) >> r) + z;
}

// Whether a m + rnd is an exact 24-bit signed multiply-add inside int32 over
// the clamped range: on each side of 0 either the multiplier is 0 (any
// truncation of a times 0 is 0) or |a| and m are below 2^23 and a m + rnd
// stays in [-2^31, 2^31) (rnd >= 0 moves negative products towards 0).
bool requant_fits24(int32_t m_pos, int32_t m_neg, int32_t a_lo, int32_t a_hi, int64_t rnd) {
  if (rnd >= (1ll << 30)) return false;
  const int64_t top = 1ll << 31, lim = 1ll << 23;
  const bool pos = m_pos == 0 || (m_pos > 0 && m_pos < lim && a_hi < lim && (int64_t)a_hi * m_pos + rnd < top);
  const bool neg = m_neg == 0 || (m_neg > 0 && m_neg < lim && -(int64_t)a_lo < lim &&
                                  -(int64_t)a_lo * m_neg - rnd <= top);
  return pos && neg;
}

// a m + rnd + z 2^r inside int32 for a in [a_lo, a_hi] (identity layers,
// m = m_pos = m_neg, 24-bit operands already checked)
bool requant_fold_fits(const LayerDev& F) {
  if (F.r < 0 || F.r > 30) return false;
  const int64_t rndz = F.rnd + (int64_t)F.z_out * (1ll << F.r);
  const int64_t lo = (int64_t)F.a_lo * F.m_pos + rndz, hi = (int64_t)F.a_hi * F.m_pos + rndz;
  const int64_t top = 1ll << 31;
  return rndz >= -top && rndz < top && lo >= -top && lo < top && hi >= -top && hi < top;
}

RqBounds requant_bounds(int32_t m_pos, int32_t m_neg, int r, int z) {
  RqBounds B;
  B.m_pos = r == 0 ? std::min<int32_t>(m_pos, 256) : m_pos;
  B.m_neg = r == 0 ? std::min<int32_t>(m_neg, 256) : m_neg;
  int64_t lo = 0, hi = INT32_MAX;
  if (requant_q(hi, B.m_pos, r, z) < 127) {
    B.a_hi = INT32_MAX;
  } else {
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (requant_q(mid, B.m_pos, r, z) >= 127) hi = mid;
      else lo = mid + 1;
    }
    B.a_hi = (int32_t)lo;
  }
  lo = INT32_MIN;
  hi = -1;
  if (requant_q(lo, B.m_neg, r, z) > -128) {
    B.a_lo = INT32_MIN;
  } else {
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (requant_q(mid, B.m_neg, r, z) <= -128) lo = mid;
      else hi = mid - 1;
    }
    B.a_lo = (int32_t)lo;
  }
  return B;
}

// Frequencies of a base depth from the counts n_s of its 255 codes (the
// integer-softmax rule with the counts in place of the exponentials):
// f_s = 1 + floor(n_s 65281 / N), N = sum n_s, and what the f_s leave of
// 2^16 goes to the lowest code of maximum count.  cdf[0] = 0, cdf[255] = 2^16.
void base_cdf(const uint32_t* n, int32_t* cdf) {
  int64_t N = 0;
  int arg = 0;
  for (int i = 0; i < 255; i++) {
    N += n[i];
    if (n[i] > n[arg]) arg = i;
  }
  if (N == 0) N = 1;
  int64_t f[255], tot = 0;
  for (int i = 0; i < 255; i++) {
    f[i] = 1 + (int64_t)n[i] * 65281 / N;
    tot += f[i];
  }
  f[arg] += 65536 - tot;
  cdf[0] = 0;
  for (int i = 0; i < 255; i++) cdf[i + 1] = cdf[i] + (int32_t)f[i];
}

struct LayerImage {
  std::vector<int8_t> packed;
  std::vector<int32_t> bias, zc;
  int ksteps, npad;
};

LayerImage build_image(const HostLayer& L) {
  LayerImage im;
  const int K = L.taps * L.cin;
  const int kpad = (int)align_up(K, 64);
  im.ksteps = kpad / 64;
  im.npad = (int)align_up(L.cout, 16);
  const int NB = im.npad / 16;
  im.packed.assign((size_t)kpad * im.npad, 0);
  for (int s = 0; s < im.ksteps; s++)
    for (int nb = 0; nb < NB; nb++)
      for (int lane = 0; lane < 64; lane++)
        for (int i = 0; i < 16; i++) {
          const int k = 64 * s + 16 * (lane / 16) + i, col = 16 * nb + lane % 16;
          int8_t v = 0;
          if (k < K && col < L.cout) v = L.W[(size_t)k * L.cout + col];
          im.packed[(((size_t)s * NB + nb) * 64 + lane) * 16 + i] = v;
        }
  im.bias.assign(im.npad, 0);
  const bool sparse = L.taps > 1;
  for (int o = 0; o < L.cout; o++) {
    int64_t b = L.bias[o];
    if (!sparse && L.z_in != 0) {
      int64_t cs = 0;
      for (int k = 0; k < K; k++) cs += L.W[(size_t)k * L.cout + o];
      b -= (int64_t)L.z_in * cs;
    }
    im.bias[o] = (int32_t)b;
  }
  if (sparse && L.z_in != 0) {
    im.zc.assign((size_t)L.taps * im.npad, 0);
    for (int t = 0; t < L.taps; t++)
      for (int o = 0; o < L.cout; o++) {
        int64_t cs = 0;
        for (int c = 0; c < L.cin; c++) cs += L.W[((size_t)t * L.cin + c) * L.cout + o];
        im.zc[(size_t)t * im.npad + o] = (int32_t)(-(int64_t)L.z_in * cs);
      }
  }
  return im;
}

}  // namespace

// ===========================================================================
// Context
// ===========================================================================
namespace {

// Grow-only device buffer carved by a bump pointer.  A measuring pass with
// base == nullptr sizes a phase before the real pass.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
  bool measuring = false;
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = (T*)(base + off);
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
};

}  // namespace

struct lpcc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;  // created when the caller passes none
  std::string err;
  char* dev[3] = {nullptr, nullptr, nullptr};  // arenas: octree, model, descriptors
  size_t cap[3] = {0, 0, 0};
  uint8_t* pinned = nullptr;  // host staging (descriptors, small read-backs)
  size_t pinned_cap = 0;
  // kernel timing
  std::string time_family;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t ev_used = 0;
  int64_t time_units = 0;
  // kernel autotuner of the GEMM-type launches, per (kernel, widths, log2
  // rows): the variant (compacted over present taps / occupied children, or
  // dense) and its tile; tiling = 0 tunes, 1/2/4 fixes the compacted
  // variants' row blocks, 11/12/14 the dense variants'
  struct TuneRec {
    int best = 0;
    int ncand = 0;
    int cand[8] = {};
    double ms[8] = {};
    int n[8] = {};
  };
  std::map<std::array<int, 5>, TuneRec> tune;
  struct Pending {
    TuneRec* rec;
    int cand;
    hipEvent_t a, z;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> ev_free;
  hipEvent_t poll_ev = nullptr;  // stream_wait's event
  int tiling = 0;
  // graph mode: every launch batch of a call is captured into a HIP graph and
  // replayed; the executable graph of each (call kind, batch) slot is kept and
  // updated in place when the next call has the same launch sequence
  int graphs = 0;
  int call_kind = 0, batch_idx = 0;
  std::map<int, hipGraphExec_t> gexec;
  int64_t graph_inst = 0, graph_upd = 0;
  // second stream of the decoder (convolutions and neighbour tables of the
  // next depth run beside the current depth's predictor and coder)
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> sync_ev;
  size_t sync_used = 0;
  // base depth B of the streams this context encodes: depths below B are
  // coded from the counts of their own codes, the model runs from depth B
  int base = 0;
  // neighbour tables: 0 = from the parent depth's table (a hash only at the
  // first convolved depth), 1 = a coordinate hash at every convolved depth
  int kmap_mode = 0;
  // workspace cap in bytes (0 = none) and the most held so far
  size_t budget = 0, peak = 0;
  // fixed mode (the entry point that allocates nothing): the arenas are
  // carved from the library's static device block, host staging is one
  // pageable buffer sized when the context is created, one stream, no events
  bool fixed = false;
  char* fixed_base = nullptr;
  size_t fixed_cap = 0, fixed_off1 = 0;
  std::unique_ptr<uint8_t[]> hostbuf;
  std::string fixed_why;        // why the static block is unavailable, if it is
  lpcc_ctx* noalloc = nullptr;  // fixed-mode companion of this context
};

namespace {

#define HIPC(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      char b_[256];                                                                  \
      snprintf(b_, sizeof(b_), "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      c->err = b_;                                                                   \
      return e_ == hipErrorOutOfMemory ? LPCC_E_NOMEM : LPCC_E_DEVICE;               \
    }                                                                                \
  } while (0)

size_t held_bytes(const lpcc_ctx* c) { return c->fixed ? 0 : c->cap[0] + c->cap[1] + c->cap[2]; }

// Fixed mode: [0, kFixedDesc) descriptors, then the octree arena, then the
// model arena of the current call, all inside the library's block.
constexpr size_t kFixedDesc = (size_t)2 << 20;

int reserve_fixed(lpcc_ctx* c, int which, size_t bytes) {
  bytes = align_up(bytes, 256);
  size_t at = which == 2 ? 0 : (which == 0 ? kFixedDesc : c->fixed_off1);
  const size_t lim = which == 2 ? kFixedDesc : c->fixed_cap;
  if (at + bytes > lim) {
    char b[256];
    snprintf(b, sizeof(b), "workspace of %zu bytes does not fit the %zu-byte static block of the allocation-free "
                           "entry point", at + bytes, which == 2 ? kFixedDesc : c->fixed_cap);
    c->err = b;
    return LPCC_E_NOMEM;
  }
  c->dev[which] = c->fixed_base + at;
  c->cap[which] = which == 2 ? kFixedDesc : bytes;
  if (which == 0) c->fixed_off1 = kFixedDesc + bytes;
  return LPCC_OK;
}

int reserve(lpcc_ctx* c, int which, size_t bytes) {
  if (c->fixed) return reserve_fixed(c, which, bytes);
  if (bytes <= c->cap[which]) return LPCC_OK;
  size_t nc = std::max(bytes, c->cap[which] + c->cap[which] / 4);
  if (c->budget) {  // grow by a quarter when the budget allows, else exactly
    const size_t others = held_bytes(c) - c->cap[which];
    if (others + nc > c->budget) nc = bytes;
    if (others + nc > c->budget) {
      char b[256];
      snprintf(b, sizeof(b), "workspace of %zu bytes over the context's budget of %zu bytes", others + nc,
               c->budget);
      c->err = b;
      return LPCC_E_NOMEM;
    }
  }
  HIPC(hipStreamSynchronize(c->stream));
  if (c->dev[which]) HIPC(hipFree(c->dev[which]));
  c->dev[which] = nullptr;
  c->cap[which] = 0;
  HIPC(hipMalloc((void**)&c->dev[which], nc));
  c->cap[which] = nc;
  c->peak = std::max(c->peak, held_bytes(c));
  return LPCC_OK;
}

int reserve_pinned(lpcc_ctx* c, size_t bytes) {
  if (bytes <= c->pinned_cap) return LPCC_OK;
  if (c->fixed) {  // the pageable buffer of the context never grows
    char b[256];
    snprintf(b, sizeof(b), "host staging of %zu bytes exceeds the %zu-byte buffer of the allocation-free entry point",
             bytes, c->pinned_cap);
    c->err = b;
    return LPCC_E_NOMEM;
  }
  size_t nc = std::max(bytes, c->pinned_cap * 2);
  HIPC(hipStreamSynchronize(c->stream));
  if (c->pinned) HIPC(hipHostFree(c->pinned));
  c->pinned = nullptr;
  c->pinned_cap = 0;
  HIPC(hipHostMalloc((void**)&c->pinned, nc, hipHostMallocDefault));
  c->pinned_cap = nc;
  return LPCC_OK;
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Descriptor batch: host bytes uploaded in one copy; launches are closures
// over offsets into the uploaded block.
struct Batch {
  lpcc_ctx* ctx = nullptr;
  bool has_events = false;  // a launch records events of its own (tuning)
  std::vector<uint8_t> bytes;
  struct L {
    std::string family;
    int64_t units;
    std::function<hipError_t(const uint8_t*)> fn;
  };
  std::vector<L> launches;
  template <class T>
  size_t add(const std::vector<T>& v) {
    size_t off = align_up(bytes.size(), 64);
    bytes.resize(off + std::max<size_t>(v.size(), 1) * sizeof(T));
    if (!v.empty()) memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
  void launch(const std::string& fam, int64_t units, std::function<hipError_t(const uint8_t*)> fn) {
    launches.push_back({fam, units, std::move(fn)});
  }
};

// Upload and enqueue a batch.  `slot` chooses the half of the descriptor
// arena so that two batches of one call never overlap.
int run_batch(lpcc_ctx* c, Batch& b, size_t* desc_off) {
  const size_t n = align_up(b.bytes.size(), 256);
  size_t need = *desc_off + n;
  if (need > c->cap[2]) {
    // everything enqueued so far, on both streams, has to finish before the
    // arena may move (an earlier batch of the call may have left work on the
    // second stream that still reads its descriptors)
    HIPC(hipStreamSynchronize(c->stream));
    if (c->side) HIPC(hipStreamSynchronize(c->side));
    *desc_off = 0;
    need = n;
    int st = reserve(c, 2, std::max<size_t>(need, 1 << 20));
    if (st) return st;
  }
  int st = reserve_pinned(c, std::max(c->pinned_cap, need));
  if (st) return st;
  // the pinned block mirrors the device block; regions of one call do not overlap
  memcpy(c->pinned + *desc_off, b.bytes.data(), b.bytes.size());
  uint8_t* dbase = (uint8_t*)c->dev[2] + *desc_off;
  const uint8_t* hsrc = c->pinned + *desc_off;
  *desc_off += n;
  const int slot = c->call_kind * 64 + c->batch_idx++;
  if (c->graphs && c->time_family.empty() && !b.has_events && !b.launches.empty()) {
    // capture the copy and the launches, then update the slot's executable
    // graph in place (same launch sequence) or instantiate a new one
    HIPC(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (!b.bytes.empty()) e = hipMemcpyAsync(dbase, hsrc, b.bytes.size(), hipMemcpyHostToDevice, c->stream);
    for (size_t k = 0; k < b.launches.size() && e == hipSuccess; k++) e = b.launches[k].fn(dbase);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    b.bytes.clear();
    b.launches.clear();
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      HIPC(e != hipSuccess ? e : e2);
    }
    bool updated = false;
    auto it = c->gexec.find(slot);
    if (it != c->gexec.end()) {
      hipGraphExecUpdateResult r;
      hipGraphNode_t en = nullptr;
      if (hipGraphExecUpdate(it->second, g, &en, &r) == hipSuccess && r == hipGraphExecUpdateSuccess) {
        updated = true;
      } else {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(it->second);
        c->gexec.erase(it);
      }
    }
    if (!updated) {
      hipGraphExec_t x = nullptr;
      const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        HIPC(ei);
      }
      c->gexec[slot] = x;
      c->graph_inst++;
    } else {
      c->graph_upd++;
    }
    (void)hipGraphDestroy(g);
    HIPC(hipGraphLaunch(c->gexec[slot], c->stream));
    return LPCC_OK;
  }
  if (!b.bytes.empty()) HIPC(hipMemcpyAsync(dbase, hsrc, b.bytes.size(), hipMemcpyHostToDevice, c->stream));
  for (auto& L : b.launches) {
    const bool timed = !c->time_family.empty() && L.family == c->time_family;
    if (timed) {
      if (c->ev_used == c->ev.size()) {
        hipEvent_t a, z;
        HIPC(hipEventCreate(&a));
        HIPC(hipEventCreate(&z));
        c->ev.push_back({a, z});
      }
      HIPC(hipEventRecord(c->ev[c->ev_used].first, c->stream));
    }
    HIPC(L.fn(dbase));
    if (timed) {
      HIPC(hipEventRecord(c->ev[c->ev_used].second, c->stream));
      c->ev_used++;
      c->time_units += L.units;
    }
  }
  b.bytes.clear();
  b.launches.clear();
  return LPCC_OK;
}

// tiles of 64 rows over a list of segments with the given row counts
std::vector<Tile> make_tiles(const std::vector<int64_t>& rows, int rows_per_tile = 64) {
  std::vector<Tile> t;
  for (size_t s = 0; s < rows.size(); s++)
    for (int64_t r = 0; r < rows[s]; r += rows_per_tile) t.push_back({(int32_t)s, (int32_t)r});
  return t;
}

int64_t nchunks_of(int64_t N, int c) { return (N + (1ll << c) - 1) >> c; }

// number of tiles make_tiles would produce (single-segment launches need only
// the count: their kernels take the segment by value)
int64_t count_tiles(const std::vector<int64_t>& rows, int rows_per_tile = 64) {
  int64_t n = 0;
  for (int64_t r : rows) n += (r + rows_per_tile - 1) / rows_per_tile;
  return n;
}

// ---- kernel autotuner ----
// Variant codes: for the 3x3x3 and other GEMM launches rb (1, 2, 4: the
// compacted gather-GEMM, or the dense one for layers without taps) or
// 10 + rb (the dense gather-GEMM over all taps); for the child convolution
// 100 + 1/2 (compacted, tiles of 64 / 128 parents) or 110 + rb (dense); for
// the upsampling 200 + 1/2 (compacted, tiles of 128 / 512 parents) or
// 210 + rb (all child slots of every parent).
struct Variant {
  int code, tile_rows;
};
std::vector<Variant> variants(bool up, int mode) {
  if (up) return {{201, 128}, {202, 512}, {211, 64}, {212, 128}, {214, 256}};
  if (mode == G_DOWN) return {{101, 64}, {102, 128}, {111, 64}, {112, 128}, {114, 256}};
  if (mode == G_CONV) return {{1, 64}, {2, 128}, {4, 256}, {11, 64}, {12, 128}, {14, 256}};
  return {{1, 64}, {2, 128}, {4, 256}};
}
// the variant a fixed tiling selects
Variant fixed_variant(bool up, int mode, int tiling, int64_t rows) {
  const bool dense = tiling > 10;
  const int rb = tiling % 10;
  if (up) {
    if (dense) return {210 + rb, 64 * rb};
    return count_tiles({rows}, 512) >= kSlotTileBlocks ? Variant{202, 512} : Variant{201, 128};
  }
  if (mode == G_DOWN) {
    if (dense) return {110 + rb, 64 * rb};
    return count_tiles({rows}, 128) >= kSlotTileBlocks ? Variant{102, 128} : Variant{101, 64};
  }
  if (mode == G_CONV) return {tiling, 64 * rb};
  return {rb, 64 * rb};
}
hipError_t launch_variant(int code, bool up, int mode, int cin, int cout, const GemmSeg* S, const Tile* T, int nt,
                          const GemmArg& one, hipStream_t st) {
  if (up) {
    if (code < 210) return launch_up_cx(cout, S, T, nt, one, code == 201 ? 128 : 512, st);
    return launch_up(cout, S, T, nt, one, code - 210, st);
  }
  if (mode == G_DOWN) {
    if (code < 110) return launch_down_cx(cout, S, T, nt, one, code == 101 ? 64 : 128, st);
    return launch_gemm_dense(mode, cin, cout, S, T, nt, one, code - 110, st);
  }
  if (code > 10) return launch_gemm_dense(mode, cin, cout, S, T, nt, one, code - 10, st);
  return launch_gemm(mode, cin, cout, S, T, nt, one, code, st);
}

hipError_t tune_event(lpcc_ctx* c, hipEvent_t* e) {
  if (!c->ev_free.empty()) {
    *e = c->ev_free.back();
    c->ev_free.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Fold finished measurements into the table; a size class is decided once
// every candidate has been timed.
void resolve_tuning(lpcc_ctx* c) {
  std::vector<lpcc_ctx::Pending> keep;
  for (auto& p : c->pending) {
    float ms = 0;
    hipError_t e = hipEventElapsedTime(&ms, p.a, p.z);
    if (e == hipErrorNotReady) {
      keep.push_back(p);
      continue;
    }
    (void)hipGetLastError();
    if (e == hipSuccess) {
      p.rec->ms[p.cand] += ms;
      p.rec->n[p.cand]++;
    }
    c->ev_free.push_back(p.a);
    c->ev_free.push_back(p.z);
  }
  c->pending.swap(keep);
  for (auto& kv : c->tune) {
    auto& r = kv.second;
    if (r.best) continue;
    int bi = -1;
    double bv = 0;
    bool all = r.ncand > 0;
    for (int k = 0; k < r.ncand; k++) {
      if (r.n[k] == 0) {
        all = false;
        break;
      }
      const double v = r.ms[k] / r.n[k];
      if (bi < 0 || v < bv) bi = k, bv = v;
    }
    if (all) r.best = r.cand[bi];
  }
}

int log2_rows(int64_t rows) {
  int b = 0;
  while ((1ll << (b + 1)) <= rows) b++;
  return b;
}

}  // namespace

// ===========================================================================
// Pipeline state of one call (all frames share every per-depth array)
// ===========================================================================
namespace {

struct Frames {
  int nf = 0;
  std::vector<std::vector<int64_t>> N;    // [f][d] nodes of frame f at depth d
  std::vector<std::vector<int64_t>> off;  // [f][d] first node of frame f at depth d
  std::vector<int64_t> tot;               // [d] nodes of all frames
};

struct Levels {
  uint64_t* key[kMaxD + 1] = {};
  uint8_t* code[kMaxD + 1] = {};
  int32_t* cstart[kMaxD + 1] = {};
};

// Model-phase buffers (depth d arrays are [tot[d]] rows)
struct ModelBufs {
  int8_t* F[kMaxD + 1] = {};         // features that predict depth d (shallow d and k0)
  int32_t* kmap[kMaxD + 1] = {};     // [28][tot[j]] for the depths that convolve: 27 taps, masks
  uint64_t* hkeys[kMaxD + 1] = {};   // hash tables: 16-byte slots {u64 key, i32 row}
  bool tree[kMaxD + 1] = {};          // neighbour table derived from depth j-1's (no hash table)
  bool hash_all = false;              // set before carving: hash every convolved depth
  int64_t tree_min = 0;               // set before carving: smaller depths hash
  uint64_t hmask[kMaxD + 1] = {};
  uint64_t* hash_lo = nullptr;        // first word of the contiguous tables
  size_t hash_words = 0;              // their extent in u64 words
  int8_t *h = nullptr, *S = nullptr;  // shallow ResBlock temporaries
  int8_t* E = nullptr;                // embedded parent codes (schedule without propagation)
  // deep temporaries per target depth d
  int8_t* G[kMaxD + 1][kMaxD + 1] = {};  // [d][j] embedding / down-sampled features at depth j
  int8_t* Gk[kMaxD + 1] = {};            // [tot[k0]][C]: G of target d at depth k0
  int8_t* dh[kMaxD + 1] = {};
  int8_t* ds[kMaxD + 1] = {};
  int8_t* Z[kMaxD + 1][kMaxD + 1] = {};  // [d][j] upsampled features at depth j (j = k0 is H)
};

constexpr int64_t kTreeMinEncode = 32768;

bool need_kmap(const lpcc_model* m, int j) { return j <= m->k0 - 1 || (j == m->k0 && m->n_deep > 0); }

// Carve the model buffers for depths in [0, last] (`wanted` selects the
// predicted depths; shallow features are always built up to min(last, k0)).
void carve_model(Arena& A, const lpcc_model* m, const Frames& fr, int last, const std::vector<bool>& wanted,
                 ModelBufs& B, int base = 0) {
  const int C = m->C, k0 = m->k0;
  const int shallow_last = std::min(last, k0);
  int64_t tmax = 0;
  for (int d = base; d <= shallow_last; d++) {
    B.F[d] = A.take<int8_t>((size_t)fr.tot[d] * C);
    tmax = std::max(tmax, fr.tot[d]);
  }
  B.h = A.take<int8_t>((size_t)tmax * C);
  B.S = A.take<int8_t>((size_t)tmax * C);
  if (!m->xfp) B.E = A.take<int8_t>((size_t)tmax * C);
  // all hash-table key arrays first and contiguous, so that one fill clears them
  const int kmax = std::min(last, k0);
  auto hashed = [&](int j) { return j >= base && need_kmap(m, j) && !(j >= last && !(j == k0 && last > k0)); };
  B.hash_lo = nullptr;
  B.hash_words = 0;
  for (int j = 0; j <= kmax; j++) {
    if (!hashed(j)) continue;  // only depths that feed a wanted depth
    // a depth whose parent depth has a neighbour table derives its own from it
    B.tree[j] = !B.hash_all && j > 0 && hashed(j - 1) && fr.tot[j] >= B.tree_min;
    if (B.tree[j]) continue;
    uint64_t sz = 1;
    while (sz < (uint64_t)std::max<int64_t>(2 * fr.tot[j], 2)) sz <<= 1;
    B.hmask[j] = sz - 1;
    B.hkeys[j] = A.take<uint64_t>(2 * sz);
    if (!B.hash_lo) B.hash_lo = B.hkeys[j];
    B.hash_words = (size_t)(B.hkeys[j] + 2 * sz - B.hash_lo);
  }
  for (int j = 0; j <= kmax; j++) {
    if (!hashed(j)) continue;
    B.kmap[j] = A.take<int32_t>((size_t)28 * fr.tot[j]);  // 27 taps + the presence masks
  }
  for (int d = k0 + 1; d <= last; d++) {
    if (!wanted[d]) continue;
    // the embedding of depth d-1 depends on the code alone: a 256-row table
    // when a child convolution reads it, rows of depth k0 otherwise
    for (int j = d - 1; j > k0; j--) B.G[d][j] = A.take<int8_t>((size_t)(j == d - 1 ? 256 : fr.tot[j]) * C);
    B.Gk[d] = A.take<int8_t>((size_t)fr.tot[k0] * C);
    B.dh[d] = A.take<int8_t>((size_t)fr.tot[k0] * C);
    B.ds[d] = A.take<int8_t>((size_t)fr.tot[k0] * C);
    for (int j = k0; j <= d; j++) B.Z[d][j] = A.take<int8_t>((size_t)fr.tot[j] * C);
  }
}

const LayerDev* dlayer(const lpcc_model* m, int d, int k) { return m->d_layers + m->first[d] + k; }

GemmSeg seg0() {
  GemmSeg s;
  memset(&s, 0, sizeof(s));
  s.split = 1 << 30;  // single input unless set
  return s;
}

// Clear every hash table of the call (one fill over the contiguous keys)
void plan_hash_clear(Batch& b, ModelBufs& B, hipStream_t st) {
  if (!B.hash_lo) return;
  uint64_t* p = B.hash_lo;
  const int64_t words = (int64_t)B.hash_words;
  b.launch("hash", 0, [=](const uint8_t*) { return launch_fill_u64(p, words, ~0ull, st); });
}

// Neighbour table of depth j from depth j-1's table, codes and first-child
// rows (the table of depth j-1 is complete)
void plan_kmap_tree(Batch& b, const Levels& lv, const Frames& fr, ModelBufs& B, int j, hipStream_t st) {
  const int64_t n = fr.tot[j], np = fr.tot[j - 1];
  const int32_t* pk = B.kmap[j - 1];
  const uint8_t* pc = lv.code[j - 1];
  const int32_t* ps = lv.cstart[j - 1];
  int32_t* km = B.kmap[j];
  b.launch("hash", n, [=](const uint8_t*) { return launch_kmap_tree(pk, np, pc, ps, km, n, st); });
}

// Hash + neighbour tables of all depths in `js` whose keys are known: one
// insertion launch and one neighbour launch for the depths that hash (tables
// cleared), then the derived tables of the others
void plan_kmaps(Batch& b, const Levels& lv, const Frames& fr, ModelBufs& B, const std::vector<int>& js,
                hipStream_t st) {
  std::vector<HashJob> jobs;
  int ib = 0, kb = 0;
  int64_t units = 0;
  for (int j : js) {
    if (!B.kmap[j] || fr.tot[j] == 0 || B.tree[j]) continue;
    HashJob h;
    memset(&h, 0, sizeof(h));
    h.keys = lv.key[j];
    h.table = B.hkeys[j];
    h.kmap = B.kmap[j];
    h.n = fr.tot[j];
    h.kstride = fr.tot[j];
    h.mask = B.hmask[j];
    h.j = j;
    h.blk_insert = ib;
    h.blk_kmap = kb;
    ib += (int)((h.n + kHashBlock - 1) / kHashBlock);
    kb += (int)((h.n + 7) / 8);  // neighbour blocks: 8 nodes each (two per wave)
    units += h.n;
    jobs.push_back(h);
  }
  if (!jobs.empty()) {
    const size_t jo = b.add(jobs);
    const int nj = (int)jobs.size();
    b.launch("hash", units, [=](const uint8_t* base) {
      return launch_hash_multi((const HashJob*)(base + jo), nj, ib, kb, st);
    });
  }
  // then the derived tables, coarse to fine (each reads the one before)
  std::vector<int> tj;
  for (int j : js)
    if (B.kmap[j] && B.tree[j]) tj.push_back(j);
  std::sort(tj.begin(), tj.end());
  for (int j : tj) plan_kmap_tree(b, lv, fr, B, j, st);
}

// Neighbour table of depth j whose hash table is already filled
void plan_kmap_only(Batch& b, const Levels& lv, const Frames& fr, ModelBufs& B, int j, hipStream_t st) {
  const int64_t n = fr.tot[j];
  const uint64_t* hk = B.hkeys[j];
  const uint64_t mask = B.hmask[j];
  int32_t* km = B.kmap[j];
  const uint64_t* keys = lv.key[j];
  b.launch("hash", n, [=](const uint8_t*) { return launch_kmap(keys, n, j, hk, mask, km, n, st); });
}

const LayerDev& hlayer(const lpcc_model* m, const LayerDev* dev) { return m->h_layers[dev - m->d_layers]; }

void plan_gemm(Batch& b, const lpcc_model* m, const char* fam, int mode, int cin, int cout,
               const std::vector<GemmSeg>& segs, hipStream_t st) {
  std::vector<int64_t> rows;
  int64_t units = 0;
  for (auto& s : segs) {
    rows.push_back(s.rows);
    units += s.rows;
  }
  if (units == 0) return;
  std::string f(fam);
  GemmArg one;
  memset(&one, 0, sizeof(one));
  size_t so = 0;
  if (segs.size() == 1) {  // by value: no descriptor loads in the kernel
    one.seg = segs[0];
    one.L = hlayer(m, segs[0].L);
    one.one = 1;
  } else {
    so = b.add(segs);
  }
  if (f == "emb") {
    const size_t to = segs.size() == 1 ? 0 : b.add(make_tiles(rows));
    const int nt = (int)count_tiles(rows);
    b.launch(f, units, [=](const uint8_t* base) {
      return launch_emb((const GemmSeg*)(base + so), (const Tile*)(base + to), nt, cout, one, st);
    });
    return;
  }
  // the variant: the tuned choice of this size class, a fixed one, or all
  // candidates timed (identical outputs: every candidate writes the same rows)
  lpcc_ctx* c = b.ctx;
  const bool up = f == "up";
  lpcc_ctx::TuneRec* rec = nullptr;
  const std::vector<Variant> all = variants(up, mode);
  std::vector<Variant> cands;
  auto of_code = [&](int code) {
    for (const Variant& v : all)
      if (v.code == code) return v;
    return all[0];
  };
  if (c->tiling) {
    cands = {fixed_variant(up, mode, c->tiling, units)};
  } else if (c->fixed) {  // no events: a decided class, else the compacted variant
    auto it = c->tune.find({up ? 1 : 0, mode, cin, cout, log2_rows(units)});
    cands = {it != c->tune.end() && it->second.best ? of_code(it->second.best) : fixed_variant(up, mode, 2, units)};
  } else {
    rec = &c->tune[{up ? 1 : 0, mode, cin, cout, log2_rows(units)}];
    if (rec->best) {
      cands = {of_code(rec->best)};
    } else {
      cands = all;
      rec->ncand = (int)all.size();
      for (size_t k = 0; k < all.size(); k++) rec->cand[k] = all[k].code;
    }
  }
  std::vector<std::pair<int, size_t>> plan;  // (variant code, tile offset)
  std::vector<int> ntiles;
  for (const Variant& v : cands) {
    plan.push_back({v.code, segs.size() == 1 ? 0 : b.add(make_tiles(rows, v.tile_rows))});
    ntiles.push_back((int)count_tiles(rows, v.tile_rows));
  }
  const bool timed = rec != nullptr && cands.size() > 1;
  if (timed) b.has_events = true;
  b.launch(f, units, [=](const uint8_t* base) {
    const GemmSeg* S = (const GemmSeg*)(base + so);
    for (size_t k = 0; k < plan.size(); k++) {
      const Tile* T = (const Tile*)(base + plan[k].second);
      auto go = [&]() { return launch_variant(plan[k].first, up, mode, cin, cout, S, T, ntiles[k], one, st); };
      if (!timed) {
        hipError_t e = go();
        if (e != hipSuccess) return e;
        continue;
      }
      hipEvent_t ea, ez;
      hipError_t e = go();  // untimed first run (code load, caches)
      if (e == hipSuccess) e = tune_event(c, &ea);
      if (e == hipSuccess) e = tune_event(c, &ez);
      if (e == hipSuccess) e = hipEventRecord(ea, st);
      if (e == hipSuccess) e = go();
      if (e == hipSuccess) e = hipEventRecord(ez, st);
      if (e != hipSuccess) return e;
      int ci = 0;
      while (rec->cand[ci] != plan[k].first) ci++;
      c->pending.push_back({rec, ci, ea, ez});
    }
    return hipSuccess;
  });
}

// Shallow depth d (1 <= d <= k0): S = ResBlock(F_{d-1}); F_d = Prune(Up([S | bits X_{d-1}])).
// The ResBlock part: on F_{d-1} with the neighbour table of depth d-1 (not
// the codes of depth d-1), or, without cross-scale propagation, on the
// embedding of the codes X_{d-1}.
void plan_shallow_convs(Batch& b, const lpcc_model* m, const Levels& lv, const Frames& fr, ModelBufs& B, int d,
                        hipStream_t st) {
  const int C = m->C;
  const int j = d - 1;
  const int rows = (int)fr.tot[j];
  const int8_t* x = B.F[j];
  int li = 0;
  if (!m->xfp) {
    GemmSeg e = seg0();
    e.code = lv.code[j];
    e.L = dlayer(m, d, li++);
    e.out = B.E;
    e.out_stride = C;
    e.rows = rows;
    plan_gemm(b, m, "emb", 0, 8, C, {e}, st);
    x = B.E;
  }
  GemmSeg s = seg0();
  s.in = x;
  s.in_stride = C;
  s.kmap = B.kmap[j];
  s.kstride = fr.tot[j];
  s.L = dlayer(m, d, li);
  s.out = B.h;
  s.out_stride = C;
  s.rows = rows;
  plan_gemm(b, m, "conv", G_CONV, C, C, {s}, st);
  s.in = B.h;
  s.L = dlayer(m, d, li + 1);
  s.out = B.S;
  s.resid = x;
  s.resid_stride = C;
  plan_gemm(b, m, "conv", G_CONV, C, C, {s}, st);
}

// Upsampling + pruning of shallow depth d (needs the codes of depth d-1)
void plan_shallow_up(Batch& b, const lpcc_model* m, const Levels& lv, const Frames& fr, ModelBufs& B, int d,
                     hipStream_t st) {
  const int C = m->C;
  const int j = d - 1;
  const int rows = (int)fr.tot[j];
  GemmSeg u = seg0();
  u.in = B.S;
  u.in_stride = C;
  u.code = lv.code[j];
  u.cstart = lv.cstart[j];
  u.L = dlayer(m, d, m->xfp ? 2 : 3);
  u.out = B.F[d];
  u.out_stride = C;
  u.rows = rows;
  u.child_rows = (int)fr.tot[d];
  plan_gemm(b, m, "up", 0, C, C, {u}, st);
}

void plan_shallow(Batch& b, const lpcc_model* m, const Levels& lv, const Frames& fr, ModelBufs& B, int d,
                  hipStream_t st) {
  plan_shallow_convs(b, m, lv, fr, B, d, st);
  plan_shallow_up(b, m, lv, fr, B, d, st);
}

// Cross-stream ordering inside a launch batch
// Waits for the work enqueued on s by polling an event instead of the
// runtime's blocking wait, so the calling thread keeps its core and the host
// code after the wait does not start on a core woken from sleep.
hipError_t stream_wait(lpcc_ctx* c, hipStream_t s) {
  if (c->fixed) return hipStreamSynchronize(s);
  if (!c->poll_ev && hipEventCreateWithFlags(&c->poll_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    c->poll_ev = nullptr;
    return hipStreamSynchronize(s);
  }
  hipError_t e = hipEventRecord(c->poll_ev, s);
  if (e != hipSuccess) return e;
  while ((e = hipEventQuery(c->poll_ev)) == hipErrorNotReady) {
  }
  return e;
}

hipEvent_t sync_event(lpcc_ctx* c) {
  if (c->sync_used == c->sync_ev.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    c->sync_ev.push_back(e);
  }
  return c->sync_ev[c->sync_used++];
}
void plan_record(Batch& b, hipEvent_t e, hipStream_t s) {
  b.launch("sync", 0, [=](const uint8_t*) { return hipEventRecord(e, s); });
}
void plan_wait(Batch& b, hipStream_t s, hipEvent_t e) {
  b.launch("sync", 0, [=](const uint8_t*) { return hipStreamWaitEvent(s, e, 0); });
}

// Deep depths `ds` (all > k0), stage by stage; every launch covers all of them.
// part 1: the re-densification (embedding and stride-2 steps; codes only),
// part 2: ResBlock at k0 and the upsampling chain (needs F_k0), 0: both.
void plan_deep(Batch& b, const lpcc_model* m, const Levels& lv, const Frames& fr, ModelBufs& B,
               const std::vector<int>& dset, hipStream_t st, int part = 0) {
  if (dset.empty()) return;
  const int C = m->C, k0 = m->k0;
  auto Gout = [&](int d, int j) -> std::pair<int8_t*, int64_t> {  // destination of depth-j G of target d
    if (j == k0) return {B.Gk[d], C};
    return {B.G[d][j], C};
  };
  if (part != 2) {
  // occupancy embedding at depth d-1
  {
    std::vector<GemmSeg> v;
    for (int d : dset) {
      GemmSeg s = seg0();
      const bool table = d - 1 > k0;  // every code's embedding (code = row)
      s.code = table ? nullptr : lv.code[d - 1];
      s.L = dlayer(m, d, 0);
      auto o = Gout(d, d - 1);
      s.out = o.first;
      s.out_stride = o.second;
      s.rows = table ? 256 : (int)fr.tot[d - 1];
      v.push_back(s);
    }
    plan_gemm(b, m, "emb", 0, 8, C, v, st);
  }
  // stride-2 steps j -> j-1 for j = d-1 .. k0+1; step t handles j = d - t
  int maxsteps = 0;
  for (int d : dset) maxsteps = std::max(maxsteps, d - 1 - k0);
  for (int t = 1; t <= maxsteps; t++) {
    std::vector<GemmSeg> v;
    for (int d : dset) {
      const int j = d - t;
      if (j <= k0) continue;
      GemmSeg s = seg0();
      s.in = B.G[d][j];
      s.in_stride = C;
      if (j == d - 1) s.ccode = lv.code[j];  // the embedding table, indexed by the child's code
      s.code = lv.code[j - 1];
      s.cstart = lv.cstart[j - 1];
      s.L = dlayer(m, d, t);
      auto o = Gout(d, j - 1);
      s.out = o.first;
      s.out_stride = o.second;
      s.rows = (int)fr.tot[j - 1];
      s.child_rows = (int)fr.tot[j];
      v.push_back(s);
    }
    plan_gemm(b, m, "down", G_DOWN, C, C, v, st);
  }
  }
  if (part == 1) return;
  // ResBlock at k0: conv1 (2C -> C), skip (2C -> C), conv2 (+ skip); without
  // cross-scale propagation conv1 (C -> C) reads G alone and the skip is G
  const bool xfp = m->xfp != 0;
  std::vector<GemmSeg> c1, sk, c2;
  for (int d : dset) {
    const int base = 1 + (d - 1 - k0);  // index of conv1 in depth d's layer list
    GemmSeg s = seg0();
    if (xfp) {
      s.in = B.F[k0];  // [F_k0 | G] without materialising the concatenation
      s.in_stride = C;
      s.in2 = B.Gk[d];
      s.in2_stride = C;
      s.split = C;
    } else {
      s.in = B.Gk[d];
      s.in_stride = C;
    }
    s.kmap = B.kmap[k0];
    s.kstride = fr.tot[k0];
    s.L = dlayer(m, d, base);
    s.out = B.dh[d];
    s.out_stride = C;
    s.rows = (int)fr.tot[k0];
    c1.push_back(s);
    GemmSeg k = seg0();
    k.in = B.F[k0];
    k.in_stride = C;
    k.in2 = B.Gk[d];
    k.in2_stride = C;
    k.split = C;
    k.L = dlayer(m, d, base + 2);
    k.out = B.ds[d];
    k.out_stride = C;
    k.rows = (int)fr.tot[k0];
    sk.push_back(k);
    GemmSeg s2 = seg0();
    s2.in = B.dh[d];
    s2.in_stride = C;
    s2.kmap = B.kmap[k0];
    s2.kstride = fr.tot[k0];
    s2.L = dlayer(m, d, base + 1);
    s2.out = B.Z[d][k0];
    s2.out_stride = C;
    s2.resid = xfp ? B.ds[d] : B.Gk[d];
    s2.resid_stride = C;
    s2.rows = (int)fr.tot[k0];
    c2.push_back(s2);
  }
  if (xfp) {
    plan_gemm(b, m, "conv", G_CONV, 2 * C, C, c1, st);
    plan_gemm(b, m, "skip", G_DENSE, 2 * C, C, sk, st);
  } else {
    plan_gemm(b, m, "conv", G_CONV, C, C, c1, st);
  }
  plan_gemm(b, m, "conv", G_CONV, C, C, c2, st);
  // upsample + prune k0 -> d
  int maxup = 0;
  for (int d : dset) maxup = std::max(maxup, d - k0);
  for (int t = 0; t < maxup; t++) {
    std::vector<GemmSeg> v;
    for (int d : dset) {
      const int j = k0 + t;
      if (j >= d) continue;
      const int base = 1 + (d - 1 - k0) + (xfp ? 3 : 2);  // first up layer
      GemmSeg u = seg0();
      u.in = B.Z[d][j];
      u.in_stride = C;
      u.code = lv.code[j];
      u.cstart = lv.cstart[j];
      u.L = dlayer(m, d, base + t);
      u.out = B.Z[d][j + 1];
      u.out_stride = C;
      u.rows = (int)fr.tot[j];
      u.child_rows = (int)fr.tot[j + 1];
      v.push_back(u);
    }
    plan_gemm(b, m, "up", 0, C, C, v, st);
  }
}

const int8_t* features_of(const lpcc_model* m, const ModelBufs& B, int d) {
  return d <= m->k0 ? B.F[d] : B.Z[d][d];
}

void plan_predict(Batch& b, const lpcc_model* m, const std::vector<PredSeg>& segs, int mode, hipStream_t st) {
  std::vector<int64_t> rows;
  int64_t units = 0;
  for (auto& s : segs) {
    rows.push_back(s.rows);
    units += s.rows;
  }
  const int nt = (int)count_tiles(rows), C = m->C;
  if (nt == 0) return;
  PredArg one;
  memset(&one, 0, sizeof(one));
  // the logit layers' requantisation: a 24-bit multiply-add with the zero
  // point in the rounding term for identity layers where that stays inside
  // int32 (2), else the general form (0)
  bool fits = true;
  for (auto& s : segs) {
    const LayerDev& F = hlayer(m, s.fc2);
    fits = fits && F.rq24 && F.m_pos == F.m_neg && requant_fold_fits(F);
  }
  one.rq24 = fits ? 2 : 0;
  size_t so = 0, to = 0;
  if (segs.size() == 1) {
    one.seg = segs[0];
    one.fc1 = hlayer(m, segs[0].fc1);
    one.fc2 = hlayer(m, segs[0].fc2);
    one.one = 1;
  } else {
    so = b.add(segs);
    to = b.add(make_tiles(rows));
  }
  const int32_t* lut = m->d_lut;
  b.launch("predict", units, [=](const uint8_t* base) {
    return launch_predict(C, mode, (const PredSeg*)(base + so), (const Tile*)(base + to), nt, lut, one, st);
  });
}

// Octree workspace of a call: staged coordinates, keys and the sort's
// digit counts, the level kernels' tile counts, and per depth the node keys,
// codes and first-child rows.  The words from `err` to the end of the sort
// counts are cleared by one fill.
struct OctreeShape {
  int nf = 0, D = 0, base = 0;
  int64_t ntot = 0;
  bool need_stage = false;
  std::vector<int64_t> ub;  // [D+1] upper bounds of the node counts
};
struct OctreeBufs {
  int32_t* xyz_stage = nullptr;
  uint64_t *kin = nullptr, *kout = nullptr;
  uint32_t *hist = nullptr, *foff = nullptr, *err = nullptr, *totals = nullptr, *bhist = nullptr;
  uint32_t *stot = nullptr, *shist = nullptr;
  char *zero_lo = nullptr, *zero_hi = nullptr;
  SortPasses sp;
  int64_t ntiles = 0, sntiles = 0;
};
constexpr int kLevelTile = 256;  // one element per thread: many blocks even for one frame

int frame_bits(int nf) {
  int b = 0;
  while ((1ll << b) < nf) b++;
  return b;
}

void carve_octree(Arena& A, const OctreeShape& S, Levels& lv, OctreeBufs& o) {
  const int D = S.D;
  o.sp = sort_passes(3 * D + frame_bits(S.nf));
  o.ntiles = (S.ntot + kLevelTile - 1) / kLevelTile;
  o.sntiles = (S.ntot + kSortTile - 1) / kSortTile;
  const size_t nbh = (size_t)S.nf * S.base * 256;
  if (S.need_stage) o.xyz_stage = A.take<int32_t>((size_t)S.ntot * 3);
  o.kin = A.take<uint64_t>(S.ntot);
  o.kout = A.take<uint64_t>(S.ntot);
  o.hist = A.take<uint32_t>((size_t)std::max<int64_t>(o.ntiles, 1) * (D + 1));
  o.foff = A.take<uint32_t>((size_t)S.nf * (D + 1));
  // zero-initialised block: error words (one per frame, one for the sort),
  // totals, base counts, code arrays, sort counts
  o.err = A.take<uint32_t>(S.nf + 1);
  o.zero_lo = (char*)o.err;
  o.totals = A.take<uint32_t>(D + 1);
  o.bhist = nbh ? A.take<uint32_t>(nbh) : nullptr;
  for (int d = 0; d <= D; d++) lv.code[d] = A.take<uint8_t>(align_up(S.ub[d], 4) + 4);
  o.stot = A.take<uint32_t>((size_t)o.sp.n * 256);
  o.shist = A.take<uint32_t>((size_t)o.sp.n * std::max<int64_t>(o.sntiles, 1) * 256);
  o.zero_hi = (char*)(o.shist + (size_t)o.sp.n * std::max<int64_t>(o.sntiles, 1) * 256);
  for (int d = 0; d <= D; d++) {
    lv.key[d] = A.take<uint64_t>(S.ub[d]);
    lv.cstart[d] = A.take<int32_t>(S.ub[d] + 1);
  }
}

OctreeShape octree_shape(int nf, const int64_t* n, int D, int base, bool need_stage) {
  OctreeShape S;
  S.nf = nf;
  S.D = D;
  S.base = base;
  S.need_stage = need_stage;
  S.ub.assign(D + 1, 0);
  for (int f = 0; f < nf; f++) {
    S.ntot += n[f];
    for (int d = 0; d <= D; d++) S.ub[d] += d >= 21 ? n[f] : std::min<int64_t>(n[f], 1ll << (3 * d));
  }
  return S;
}

// Octree of all frames: Morton keys, radix sort, level arrays.  Fills
// `fr` (after a synchronisation) and the level pointers.
int build_octree(lpcc_ctx* c, const lpcc_model* m, int nf, const int32_t* const* xyz, const int64_t* n,
                 Levels& lv, Frames& fr, std::vector<int>& fstatus, size_t* desc_off, int base = 0,
                 std::vector<uint32_t>* base_hist = nullptr) {
  const int D = m->D;
  hipStream_t st = c->stream;
  std::vector<int64_t> start(nf + 1, 0);
  for (int f = 0; f < nf; f++) start[f + 1] = start[f] + n[f];
  const int64_t ntot = start[nf];
  if (3 * D + frame_bits(nf) > 64) {
    c->err = "too many frames for this depth";
    return LPCC_E_INVAL;
  }
  bool need_stage = false;
  for (int f = 0; f < nf; f++)
    if (n[f] > 0 && !is_device_ptr(xyz[f])) need_stage = true;
  const OctreeShape S = octree_shape(nf, n, D, base, need_stage);
  const size_t nbh = (size_t)nf * base * 256;  // code counts of the base depths
  OctreeBufs o;
  Arena meas;
  carve_octree(meas, S, lv, o);
  int s = reserve(c, 0, meas.off + 4096);
  if (s) return s;
  Arena A;
  A.base = c->dev[0];
  A.cap = c->cap[0];
  carve_octree(A, S, lv, o);
  uint32_t *err = o.err, *hist = o.hist, *totals = o.totals, *foff = o.foff, *bhist = o.bhist;

  HIPC(launch_fill_u32(foff, (int64_t)nf * (D + 1), 0xFFFFFFFFu, st));
  HIPC(launch_fill_u32((uint32_t*)o.zero_lo, (int64_t)(align_up((size_t)(o.zero_hi - o.zero_lo), 4) / 4), 0, st));
  // coordinates on the device (host frames staged), then the keys of up to
  // kMortonGroup frames per launch with the first pass's digit counts
  std::vector<const int32_t*> src(nf, nullptr);
  for (int f = 0; f < nf; f++) {
    if (n[f] <= 0) continue;
    src[f] = xyz[f];
    if (!is_device_ptr(src[f])) {
      HIPC(hipMemcpyAsync(o.xyz_stage + 3 * start[f], xyz[f], (size_t)n[f] * 12, hipMemcpyHostToDevice, st));
      src[f] = o.xyz_stage + 3 * start[f];
    }
  }
  for (int f0 = 0; f0 < nf; f0 += kMortonGroup) {
    MortonFrames mf;
    memset(&mf, 0, sizeof(mf));
    mf.nf = std::min(kMortonGroup, nf - f0);
    mf.f0 = f0;
    for (int g = 0; g <= mf.nf; g++) mf.start[g] = start[f0 + g];
    for (int g = 0; g < mf.nf; g++) mf.xyz[g] = src[f0 + g];
    HIPC(launch_morton_sort0(mf, D, o.kin, err, o.sp, o.shist, o.stot, st));
  }
  uint64_t* sorted = o.kin;
  if (ntot > 0) {
    uint64_t *a = o.kin, *b = o.kout;
    for (int p = 0; p < o.sp.n; p++) {
      HIPC(launch_sort_pass(a, b, ntot, o.sp, p, o.shist, o.stot, err + nf, st));
      std::swap(a, b);
    }
    sorted = a;
    const int tile = kLevelTile;
    HIPC(launch_level_hist(sorted, ntot, D, tile, hist, st));
    HIPC(launch_level_scan(hist, (int)o.ntiles, D, totals, st));
    LevelOut lo;
    memset(&lo, 0, sizeof(lo));
    for (int d = 0; d <= D; d++) {
      lo.key[d] = lv.key[d];
      lo.code[d] = lv.code[d];
      lo.cstart[d] = lv.cstart[d];
    }
    lo.frame_off = foff;
    HIPC(launch_level_write(sorted, ntot, D, tile, hist, totals, lo, st));
    if (nbh) {
      // code counts per (frame, base depth); the node counts are still on
      // the device, so the range covers the upper bounds and the kernel
      // skips entries beyond the real count of their depth
      BaseLevels bl;
      memset(&bl, 0, sizeof(bl));
      bl.nb = base;
      bl.nf = nf;
      bl.count = totals;
      for (int d = 0; d < base; d++) {
        bl.key[d] = lv.key[d];
        bl.code[d] = lv.code[d];
        bl.start[d + 1] = bl.start[d] + S.ub[d];
      }
      HIPC(launch_base_hist(bl, bhist, st));
    }
  }
  // read back frame offsets, errors, counts (and the base depths' code
  // counts) in one copy: they were carved one after another
  const bool with_bh = nbh && ntot > 0;
  const char* rb0 = (const char*)foff;
  const char* rb1 = with_bh ? (const char*)(bhist + nbh) : (const char*)(totals + D + 1);
  const size_t rb = (size_t)(rb1 - rb0);
  s = reserve_pinned(c, *desc_off + align_up(rb, 256) + 256);
  if (s) return s;
  char* h8 = (char*)(c->pinned + c->pinned_cap - align_up(rb, 256));
  HIPC(hipMemcpyAsync(h8, rb0, rb, hipMemcpyDeviceToHost, st));
  HIPC(stream_wait(c, st));
  const uint32_t* h_foff = (const uint32_t*)h8;
  const uint32_t* h_err = (const uint32_t*)(h8 + ((const char*)err - rb0));
  if (h_err[nf] & ERR_SORT) {
    c->err = "radix sort produced an impossible rank";
    return LPCC_E_DEVICE;
  }
  const uint32_t* h_tot = (const uint32_t*)(h8 + ((const char*)totals - rb0));
  if (base_hist) {
    base_hist->assign(nbh, 0u);
    if (with_bh) memcpy(base_hist->data(), h8 + ((const char*)bhist - rb0), nbh * 4);
  }
  fr.nf = nf;
  fr.tot.assign(D + 1, 0);
  for (int d = 0; d <= D; d++) fr.tot[d] = h_tot[d];
  fr.N.assign(nf, std::vector<int64_t>(D + 1, 0));
  fr.off.assign(nf, std::vector<int64_t>(D + 1, 0));
  fstatus.assign(nf, LPCC_OK);
  for (int f = 0; f < nf; f++)
    if (h_err[f] & ERR_COORD) fstatus[f] = LPCC_E_INVAL;
  for (int d = 0; d <= D; d++) {
    int64_t next = fr.tot[d];
    for (int f = nf - 1; f >= 0; f--) {
      const uint32_t o = h_foff[f * (D + 1) + d];
      if (n[f] <= 0 || o == 0xFFFFFFFFu) {
        fr.off[f][d] = next;
        fr.N[f][d] = 0;
        continue;
      }
      fr.off[f][d] = o;
      fr.N[f][d] = next - o;
      next = o;
    }
  }
  return LPCC_OK;
}

}  // namespace

// ===========================================================================
// Encode (and level_probs) of a batch of frames
// ===========================================================================
namespace {

struct OutSpec {
  uint8_t* const* out;
  const size_t* cap;
  size_t* out_len;
};

// Header bytes of the base tables per frame: B, then per depth m and m
// (code, count) pairs of the codes present.
std::vector<size_t> base_table_bytes(const std::vector<uint32_t>& bhist, int nf, int nb) {
  std::vector<size_t> t(nf, 0);
  for (int f = 0; f < nf && nb > 0; f++) {
    t[f] = 1;
    for (int d = 0; d < nb; d++) {
      t[f] += 1;
      for (int k = 1; k < 256; k++) t[f] += bhist.empty() || bhist[((size_t)f * nb + d) * 256 + k] ? 5 : 0;
    }
  }
  return t;
}

// Chunk table, coder scratch and per-frame output staging of an encode call
struct EncLayout {
  std::vector<Chunk> chunks;
  std::vector<int> chunk_frame;
  int64_t scratch_bytes = 0;
  std::vector<size_t> stage_off;
  size_t stage_bytes = 0;
  std::vector<int64_t> dbase;  // [D+1] first node of every depth in the per-call node arrays
};

EncLayout enc_layout(const Frames& fr, int D, int cl, bool probe, const std::vector<size_t>& tbytes) {
  EncLayout L;
  const int nf = fr.nf;
  L.dbase.assign(D + 1, 0);
  for (int d = 0; d < D; d++) L.dbase[d + 1] = L.dbase[d] + fr.tot[d];
  L.stage_off.assign(nf, 0);
  if (probe) return L;
  size_t nch_all = 0;
  for (int f = 0; f < nf; f++)
    for (int d = 0; d < D; d++) nch_all += (size_t)nchunks_of(fr.N[f][d], cl);
  L.chunks.reserve(nch_all);
  L.chunk_frame.reserve(nch_all);
  for (int f = 0; f < nf; f++)
    for (int d = 0; d < D; d++) {
      const int64_t Nfd = fr.N[f][d];
      for (int64_t k = 0; k < nchunks_of(Nfd, cl); k++) {
        Chunk ch;
        ch.node0 = L.dbase[d] + fr.off[f][d] + (k << cl);
        ch.count = (int32_t)std::min<int64_t>(1ll << cl, Nfd - (k << cl));
        ch.pad_ = 0;
        ch.scratch = L.scratch_bytes;
        L.scratch_bytes += align_up(2 * (size_t)ch.count + 16, 16);
        L.chunks.push_back(ch);
        L.chunk_frame.push_back(f);
      }
    }
  // per-frame output staging (host outputs and frames that fail): header
  // bound + the frame's chunk scratch bound
  std::vector<size_t> fbytes(nf, 16 + 4 * (size_t)D);
  for (int f = 0; f < nf; f++) fbytes[f] += tbytes[f];
  for (size_t k = 0; k < L.chunks.size(); k++)
    fbytes[L.chunk_frame[k]] += 2 + align_up(2 * (size_t)L.chunks[k].count + 16, 16);
  for (int f = 0; f < nf; f++) {
    L.stage_off[f] = L.stage_bytes;
    L.stage_bytes += align_up(fbytes[f], 256);
  }
  return L;
}

struct EncBufs {
  uint32_t* sf = nullptr;
  int32_t* cdf_stage = nullptr;
  uint8_t* scratch = nullptr;
  uint32_t* lens = nullptr;
  uint8_t* stage = nullptr;
};

void carve_encode(Arena& A, const lpcc_model* m, const Frames& fr, int last, const std::vector<bool>& wanted, int nb,
                  int probe_level, bool cdf_dev, const EncLayout& L, ModelBufs& B, EncBufs& o) {
  carve_model(A, m, fr, last, wanted, B, nb);
  if (probe_level < 0) {
    o.sf = A.take<uint32_t>(L.dbase[m->D]);
    o.scratch = A.take<uint8_t>(L.scratch_bytes);
    o.lens = A.take<uint32_t>(L.chunks.size());
    o.stage = A.take<uint8_t>(L.stage_bytes);
  } else if (!cdf_dev) {
    o.cdf_stage = A.take<int32_t>((size_t)fr.tot[probe_level] * 256);
  }
}

// Descriptor bytes a call may upload: segment and tile tables, chunk tables
// and headers stay far below this bound.
size_t desc_bound(const Frames& fr, size_t nch) {
  int64_t rows = 0;
  for (int64_t t : fr.tot) rows += t;
  return ((size_t)1 << 20) + 16 * (size_t)rows + 64 * nch;
}

// Frames whose node counts are the upper bounds of an encode of n[f] points
Frames bound_frames(int nf, const int64_t* n, int D) {
  Frames fr;
  fr.nf = nf;
  fr.tot.assign(D + 1, 0);
  fr.N.assign(nf, std::vector<int64_t>(D + 1, 0));
  fr.off.assign(nf, std::vector<int64_t>(D + 1, 0));
  for (int f = 0; f < nf; f++)
    for (int d = 0; d <= D; d++) {
      fr.N[f][d] = d >= 21 ? n[f] : std::min<int64_t>(n[f], 1ll << (3 * d));
      fr.off[f][d] = fr.tot[d];
      fr.tot[d] += fr.N[f][d];
    }
  return fr;
}

}  // namespace

// Upper bounds of the three arenas an encode of these frames needs (the
// node count of every depth at its largest: min(points, 8^d); every depth
// modelled, which needs the most).
void lpcc::encode_workspace_bound(const lpcc_model* m, int nf, const int64_t* n, int cl, bool host_in,
                                  size_t out[3]) {
  const int D = m->D, nb = 0;
  const OctreeShape S = octree_shape(nf, n, D, nb, host_in);
  Levels lv;
  OctreeBufs o;
  Arena a0;
  carve_octree(a0, S, lv, o);
  const Frames fr = bound_frames(nf, n, D);
  std::vector<uint32_t> none;
  const EncLayout EL = enc_layout(fr, D, cl, false, base_table_bytes(none, nf, nb));
  std::vector<bool> wanted(D, true);
  for (int d = 0; d < nb && d < D; d++) wanted[d] = false;
  ModelBufs B;
  // the bound counts a hash table at every convolved depth: an encode
  // hashes the depths below kTreeMinEncode nodes, and the bound's node
  // counts are upper bounds
  B.hash_all = true;
  EncBufs eb;
  Arena a1;
  carve_encode(a1, m, fr, D - 1, wanted, nb, -1, false, EL, B, eb);
  out[0] = a0.off + 4096;
  out[1] = a1.off + 4096;
  out[2] = desc_bound(fr, EL.chunks.size());
}

namespace {

int encode_impl(lpcc_ctx* c, const lpcc_model* m, int nf, const int32_t* const* xyz, const int64_t* n, int cl,
                OutSpec os, int* status, int probe_level, int32_t* cdf_out, int64_t cdf_cap, int64_t* n_nodes) {
  const int D = m->D, C = m->C, k0 = m->k0;
  resolve_tuning(c);
  c->call_kind = probe_level >= 0 ? 2 : 0;
  c->batch_idx = 0;
  hipStream_t st = c->stream;
  size_t desc_off = 0;
  Levels lv;
  Frames fr;
  std::vector<int> fst;
  // base depth: depths below it are coded from their own code counts
  const int nb = probe_level >= 0 ? 0 : c->base;
  if (nb > k0) {
    c->err = "base depth above the dense fusion depth of the model";
    for (int g = 0; g < nf; g++) status[g] = LPCC_E_INVAL;
    return LPCC_E_INVAL;
  }
  std::vector<uint32_t> bhist;
  int s = build_octree(c, m, nf, xyz, n, lv, fr, fst, &desc_off, nb, &bhist);
  if (s) return s;
  for (int f = 0; f < nf; f++)
    if (fst[f] != LPCC_OK) {
      for (int g = 0; g < nf; g++) status[g] = fst[g];
      return fst[f];
    }
  const bool probe = probe_level >= 0;
  const int last = probe ? probe_level : D - 1;
  std::vector<bool> wanted(D, !probe);
  if (probe) wanted[probe_level] = true;
  for (int d = 0; d < nb; d++) wanted[d] = false;
  // static tables of the base depths: int32 CDF per (frame, depth)
  std::vector<int32_t> bcdf((size_t)nf * nb * 256, 0);
  for (int f = 0; f < nf; f++)
    for (int d = 0; d < nb; d++) {
      const size_t t = ((size_t)f * nb + d) * 256;
      base_cdf(bhist.data() + t + 1, bcdf.data() + t);  // counts of codes 1..255
    }
  if (probe) {
    *n_nodes = fr.tot[probe_level];
    if (fr.tot[probe_level] > cdf_cap) {
      status[0] = LPCC_E_CAPACITY;
      return LPCC_E_CAPACITY;
    }
  }
  // ---- model phase buffers
  std::vector<size_t> tbytes = base_table_bytes(bhist, nf, nb);
  const EncLayout EL = enc_layout(fr, D, cl, probe, tbytes);
  const std::vector<Chunk>& chunks = EL.chunks;
  const std::vector<int>& chunk_frame = EL.chunk_frame;
  const std::vector<int64_t>& dbase = EL.dbase;
  const std::vector<size_t>& stage_off = EL.stage_off;
  const bool cdf_dev = probe && is_device_ptr(cdf_out);
  ModelBufs B;
  B.hash_all = c->kmap_mode == 1;
  // the encoder hashes every depth it can in two launches; a derived table
  // costs a launch of its own, which pays from about this many nodes
  B.tree_min = kTreeMinEncode;
  EncBufs eb;
  Arena meas;
  carve_encode(meas, m, fr, last, wanted, nb, probe ? probe_level : -1, cdf_dev, EL, B, eb);
  s = reserve(c, 1, meas.off + 4096);
  if (s) return s;
  Arena A;
  A.base = c->dev[1];
  A.cap = c->cap[1];
  carve_encode(A, m, fr, last, wanted, nb, probe ? probe_level : -1, cdf_dev, EL, B, eb);
  uint32_t* sf = eb.sf;
  int32_t* cdf_stage = eb.cdf_stage;
  uint8_t* scratch = eb.scratch;
  uint32_t* lens = eb.lens;
  uint8_t* stage = eb.stage;

  Batch b;
  b.ctx = c;
  // F_B = 0: the first modelled depth has no coarser context
  {
    int8_t* f0 = B.F[nb];
    const int64_t bytes = fr.tot[nb] * C;
    b.launch("fill", 0, [=](const uint8_t*) { return launch_fill_u32((uint32_t*)f0, (bytes + 3) / 4, 0, st); });
  }
  {
    std::vector<int> js;
    for (int j = nb; j <= std::min(last, k0); j++)
      if (B.kmap[j]) js.push_back(j);
    plan_hash_clear(b, B, st);
    plan_kmaps(b, lv, fr, B, js, st);
  }
  // start/freq of every base node from its frame's table
  if (nb > 0 && dbase[nb] > 0) {
    BaseLevels bl;
    memset(&bl, 0, sizeof(bl));
    bl.nb = nb;
    bl.nf = nf;
    for (int d = 0; d < nb; d++) {
      bl.key[d] = lv.key[d];
      bl.code[d] = lv.code[d];
      bl.start[d + 1] = dbase[d + 1];
    }
    const size_t to = b.add(bcdf);
    uint32_t* sf0 = sf;
    b.launch("base", dbase[nb], [=](const uint8_t* base) {
      return launch_base_sf(bl, (const int32_t*)(base + to), sf0, st);
    });
  }
  // The GPU waits for nothing but these launches: submit them, so that it
  // builds the tables while the model stages are planned and launched.
  if (!c->graphs) {
    s = run_batch(c, b, &desc_off);
    if (s) return s;
  }
  // Two streams: the re-densification of the deep depths needs only the
  // codes and runs beside the shallow chain; the predictor of the shallow
  // depths runs beside the deep ResBlock and upsampling.
  c->sync_used = 0;
  bool two = c->time_family.empty() && !c->graphs && !c->fixed;
  if (two && !c->side && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    c->side = nullptr;
  }
  two = two && c->side;
  const hipStream_t sd = two ? c->side : st;
  bool ok_ev = true;
  auto mark = [&](hipStream_t ss) -> hipEvent_t {
    if (!two) return nullptr;
    hipEvent_t e = sync_event(c);
    if (!e) {
      ok_ev = false;
      return nullptr;
    }
    plan_record(b, e, ss);
    return e;
  };
  auto wait = [&](hipStream_t ss, hipEvent_t e) {
    if (two && e) plan_wait(b, ss, e);
  };
  std::vector<int> dset;
  for (int d = k0 + 1; d <= last; d++)
    if (wanted[d]) dset.push_back(d);
  wait(sd, mark(st));  // the side stream starts after the fills
  plan_deep(b, m, lv, fr, B, dset, sd, 1);
  hipEvent_t g_done = mark(sd);
  // the re-densification is long GPU work: submit it before planning the
  // rest (the next batch's first side-stream launch waits for an event the
  // main stream records after that batch's descriptors are copied)
  if (!c->graphs) {
    if (!ok_ev) {
      c->err = "event creation failed";
      return LPCC_E_DEVICE;
    }
    s = run_batch(c, b, &desc_off);
    if (s) return s;
  }
  for (int d = nb + 1; d <= std::min(last, k0); d++) plan_shallow(b, m, lv, fr, B, d, st);
  hipEvent_t f_done = mark(st);
  wait(st, g_done);
  plan_deep(b, m, lv, fr, B, dset, st, 2);
  // predictor: shallow depths on the side stream, deep depths here
  std::vector<PredSeg> ps, pd;
  for (int d = 0; d <= last; d++) {
    if (!wanted[d] || fr.tot[d] == 0) continue;
    PredSeg p;
    memset(&p, 0, sizeof(p));
    p.F = features_of(m, B, d);
    p.code = lv.code[d];
    p.fc1 = dlayer(m, d, m->first[d + 1] - m->first[d] - 2);
    p.fc2 = dlayer(m, d, m->first[d + 1] - m->first[d] - 1);
    p.rows = (int)fr.tot[d];
    if (probe) p.cdf32 = cdf_dev ? cdf_out : cdf_stage;
    else p.sf = sf + dbase[d];
    (d <= k0 && two ? ps : pd).push_back(p);
  }
  if (!ps.empty()) {
    wait(sd, f_done);
    plan_predict(b, m, ps, probe ? 2 : 0, sd);
  }
  plan_predict(b, m, pd, probe ? 2 : 0, st);
  wait(st, mark(sd));
  if (!ok_ev) {
    c->err = "event creation failed";
    return LPCC_E_DEVICE;
  }
  // ---- stream layout: header (fixed part, then one 16-bit length per
  // chunk), then the payloads in chunk order
  const size_t nch = chunks.size();
  std::vector<size_t> nchf(nf, 0), first(nf, 0), hpre(nf, 0);
  for (size_t k = 0; k < nch; k++) nchf[chunk_frame[k]]++;
  for (int f = 1; f < nf; f++) first[f] = first[f - 1] + nchf[f - 1];
  // header of frame f; the chunk lengths are filled in when hl is given
  auto make_header = [&](int f, const uint32_t* hl) {
    std::vector<uint8_t> H;
    const size_t pre = 16 + 4 * (size_t)D + tbytes[f];
    hpre[f] = pre;
    H.assign(pre + 2 * nchf[f], 0);
    H[0] = 'L'; H[1] = 'P'; H[2] = 'C'; H[3] = '1';
    H[4] = nb > 0 ? 2 : 1; H[5] = (uint8_t)D; H[6] = (uint8_t)m->n_deep; H[7] = (uint8_t)cl;
    auto w32 = [&](size_t o, uint32_t v) { for (int k = 0; k < 4; k++) H[o + k] = (uint8_t)(v >> (8 * k)); };
    w32(8, m->blob_id);
    w32(12, (uint32_t)fr.N[f][D]);
    for (int d = 0; d < D; d++) w32(16 + 4 * d, (uint32_t)fr.N[f][d]);
    if (nb > 0) {  // B, then per base depth the (code, count) pairs of its present codes
      size_t o = 16 + 4 * (size_t)D;
      H[o++] = (uint8_t)nb;
      for (int d = 0; d < nb; d++) {
        const uint32_t* cnt = bhist.data() + ((size_t)f * nb + d) * 256;
        int mcodes = 0;
        for (int k = 1; k < 256; k++) mcodes += cnt[k] ? 1 : 0;
        H[o++] = (uint8_t)mcodes;
        for (int k = 1; k < 256; k++)
          if (cnt[k]) {
            H[o] = (uint8_t)k;
            w32(o + 1, cnt[k]);
            o += 5;
          }
      }
    }
    if (hl)
      for (size_t k = 0; k < nchf[f]; k++) {
        H[pre + 2 * k] = (uint8_t)(hl[first[f] + k] & 0xFF);
        H[pre + 2 * k + 1] = (uint8_t)(hl[first[f] + k] >> 8);
      }
    return H;
  };
  // Device outputs: the payloads and the length table are placed on the
  // device right after the coder, and the header's fixed part travels in the
  // descriptor block, so no host round trip separates coding and placement.
  bool on_dev = !probe && nch > 0;
  for (int f = 0; f < nf && on_dev; f++) on_dev = is_device_ptr(os.out[f]);
  uint32_t* hlens = nullptr;  // chunk lengths in pinned memory (device-output path)
  std::vector<std::vector<uint8_t>> hdr(nf);
  if (!probe && nch > 0) {
    const size_t co = b.add(chunks);
    const int n_ch = (int)nch;
    b.launch("rc_encode", dbase[D], [=](const uint8_t* base) {
      return launch_rc_encode((const Chunk*)(base + co), n_ch, sf, scratch, lens, st);
    });
    if (on_dev) {
      std::vector<PackFrame> pf(nf);
      std::vector<int32_t> fof(chunk_frame.begin(), chunk_frame.end());
      std::vector<uint8_t> hblob;
      std::vector<size_t> hoff(nf, 0);
      for (int f = 0; f < nf; f++) {
        hdr[f] = make_header(f, nullptr);
        pf[f].out = os.out[f];
        pf[f].cap = (uint64_t)os.cap[f];
        pf[f].first = (uint32_t)first[f];
        pf[f].pre = (uint32_t)hpre[f];
        pf[f].hsz = hdr[f].size();
        hoff[f] = hblob.size();
        hblob.insert(hblob.end(), hdr[f].begin(), hdr[f].begin() + hpre[f]);
        hblob.resize(align_up(hblob.size(), 16), 0);
      }
      const size_t fo = b.add(fof), pfo = b.add(pf), ho = b.add(hblob);
      b.launch("pack", 0, [=](const uint8_t* base) {
        return launch_rc_pack_dev((const Chunk*)(base + co), n_ch, (const int32_t*)(base + fo),
                                  (const PackFrame*)(base + pfo), scratch, lens, st);
      });
      for (int f = 0; f < nf; f++) {
        uint8_t* o = os.out[f];
        const size_t at = ho + hoff[f], n_ = std::min<size_t>(hpre[f], (size_t)os.cap[f]);
        if (n_ == 0) continue;
        b.launch("header", 0, [=](const uint8_t* base) {
          return hipMemcpyAsync(o, base + at, n_, hipMemcpyDeviceToDevice, st);
        });
      }
      // the lengths come back with the same batch, for the totals
      const size_t lb = align_up(nch * 4, 256);
      s = reserve_pinned(c, desc_off + align_up(b.bytes.size(), 256) + lb);
      if (s) return s;
      hlens = (uint32_t*)(c->pinned + c->pinned_cap - lb);
      uint32_t* hl_ = hlens;
      const uint32_t* dl = lens;
      const size_t nb_ = nch * 4;
      b.launch("lens", 0, [=](const uint8_t*) { return hipMemcpyAsync(hl_, dl, nb_, hipMemcpyDeviceToHost, st); });
    }
  }
  s = run_batch(c, b, &desc_off);
  if (s) return s;

  if (probe) {
    if (!cdf_dev && fr.tot[probe_level] > 0)
      HIPC(hipMemcpyAsync(cdf_out, cdf_stage, (size_t)fr.tot[probe_level] * 1024, hipMemcpyDeviceToHost, st));
    HIPC(stream_wait(c, st));
    status[0] = LPCC_OK;
    return LPCC_OK;
  }
  if (on_dev) {
    HIPC(stream_wait(c, st));
    int ret = LPCC_OK;
    for (int f = 0; f < nf; f++) {
      size_t total = hdr[f].size();
      for (size_t k = 0; k < nchf[f]; k++) total += hlens[first[f] + k];
      os.out_len[f] = total;
      status[f] = total > os.cap[f] ? LPCC_E_CAPACITY : LPCC_OK;
      if (status[f] != LPCC_OK && ret == LPCC_OK) ret = status[f];
    }
    return ret;
  }

  // ---- host outputs (or none): lengths first, then headers and placement
  std::vector<uint32_t> hl(nch);
  if (nch) {  // through pinned memory, past this call's descriptor blocks
    const size_t lb = align_up(nch * 4, 256);
    s = reserve_pinned(c, desc_off + lb);
    if (s) return s;
    uint32_t* hp = (uint32_t*)(c->pinned + c->pinned_cap - lb);
    HIPC(hipMemcpyAsync(hp, lens, nch * 4, hipMemcpyDeviceToHost, st));
    HIPC(stream_wait(c, st));
    memcpy(hl.data(), hp, nch * 4);
  }
  std::vector<size_t> total(nf, 0);
  std::vector<uint8_t*> dst(nch, nullptr);
  std::vector<bool> odev(nf, false);
  for (int f = 0; f < nf; f++) {
    hdr[f] = make_header(f, hl.data());
    size_t pay = 0;
    for (size_t k = 0; k < nchf[f]; k++) pay += hl[first[f] + k];
    total[f] = hdr[f].size() + pay;
    os.out_len[f] = total[f];
    status[f] = total[f] > os.cap[f] ? LPCC_E_CAPACITY : LPCC_OK;
    odev[f] = is_device_ptr(os.out[f]);
  }
  for (int f = 0; f < nf; f++) {
    const bool direct = status[f] == LPCC_OK && odev[f];
    uint8_t* base = direct ? os.out[f] : stage + stage_off[f];
    size_t o = hdr[f].size();
    for (size_t k = 0; k < nchf[f]; k++) {
      dst[first[f] + k] = base + o;
      o += hl[first[f] + k];
    }
  }
  // payload placement and the headers of device outputs in one batch: the
  // headers travel with the descriptor block and are copied on the device
  if (nch) {
    const size_t co = b.add(chunks), po = b.add(dst);
    const int n_ch = (int)nch;
    b.launch("pack", 0, [=](const uint8_t* base) {
      return launch_rc_pack((const Chunk*)(base + co), n_ch, scratch, lens, (uint8_t* const*)(base + po), st);
    });
  }
  {
    std::vector<uint8_t> hblob;
    std::vector<size_t> hoff(nf, 0);
    for (int f = 0; f < nf; f++) {
      if (status[f] != LPCC_OK || !odev[f]) continue;
      hoff[f] = hblob.size();
      hblob.insert(hblob.end(), hdr[f].begin(), hdr[f].end());
      hblob.resize(align_up(hblob.size(), 16), 0);
    }
    if (!hblob.empty()) {
      const size_t ho = b.add(hblob);
      for (int f = 0; f < nf; f++) {
        if (status[f] != LPCC_OK || !odev[f]) continue;
        uint8_t* o = os.out[f];
        const size_t at = ho + hoff[f], n_ = hdr[f].size();
        b.launch("header", 0, [=](const uint8_t* base) {
          return hipMemcpyAsync(o, base + at, n_, hipMemcpyDeviceToDevice, st);
        });
      }
    }
  }
  if (!b.launches.empty()) {
    s = run_batch(c, b, &desc_off);
    if (s) return s;
  }
  for (int f = 0; f < nf; f++) {
    if (status[f] != LPCC_OK) continue;
    if (!odev[f]) {
      memcpy(os.out[f], hdr[f].data(), hdr[f].size());
      if (total[f] > hdr[f].size())
        HIPC(hipMemcpyAsync(os.out[f] + hdr[f].size(), stage + stage_off[f] + hdr[f].size(),
                            total[f] - hdr[f].size(), hipMemcpyDeviceToHost, st));
    }
  }
  HIPC(stream_wait(c, st));
  int ret = LPCC_OK;
  for (int f = 0; f < nf; f++)
    if (status[f] != LPCC_OK && ret == LPCC_OK) ret = status[f];
  return ret;
}

}  // namespace

// ===========================================================================
// Decode of a batch of frames
// ===========================================================================
namespace {

struct Header {
  int D = 0, n_deep = 0, cl = 0;
  int B = 0;                  // base depth (version 2), 0 in version 1
  uint32_t blob = 0;
  std::vector<int64_t> N;     // [D+1]
  std::vector<uint32_t> cnt;  // [B][255] counts of codes 1..255 per base depth
  std::vector<uint32_t> len;  // chunk lengths
  size_t pre = 0;             // offset of the chunk lengths
  size_t hdr = 0, total = 0;
  size_t bound = 0;           // header bytes that certainly suffice (when hdr is not known yet)
};

// Parse a stream header from the `avail` bytes at h (the stream has `len`).
// LPCC_E_CAPACITY: more bytes are needed (H.bound, or H.hdr once known).
int parse_header(const uint8_t* h, size_t avail, size_t len, Header& H, bool need_lengths) {
  if (len < 16 || avail < 16) return LPCC_E_CORRUPT;
  if (h[0] != 'L' || h[1] != 'P' || h[2] != 'C' || h[3] != '1' || (h[4] != 1 && h[4] != 2)) return LPCC_E_CORRUPT;
  H.D = h[5];
  H.n_deep = h[6];
  H.cl = h[7];
  H.blob = rd32(h + 8);
  if (H.D < 1 || H.D > kMaxD || H.cl < 4 || H.cl > 14) return LPCC_E_CORRUPT;
  const size_t fixed = 16 + 4 * (size_t)H.D;
  if (len < fixed) return LPCC_E_CORRUPT;
  H.hdr = 0;
  H.bound = len;
  if (avail < fixed) return LPCC_E_CAPACITY;  // caller fetches more
  H.N.assign(H.D + 1, 0);
  H.N[H.D] = rd32(h + 12);
  for (int d = 0; d < H.D; d++) H.N[d] = rd32(h + 16 + 4 * d);
  if (H.N[0] > 1 || ((H.N[0] == 0) != (H.N[H.D] == 0))) return LPCC_E_CORRUPT;
  for (int d = 0; d < H.D; d++)
    if (H.N[d + 1] < H.N[d] || H.N[d + 1] > 8 * H.N[d]) return LPCC_E_CORRUPT;
  int64_t nch = 0;
  for (int d = 0; d < H.D; d++) nch += nchunks_of(H.N[d], H.cl);
  size_t pre = fixed;
  H.B = 0;
  H.cnt.clear();
  H.bound = fixed + 1 + (size_t)(H.D - 1) * (1 + 5 * 255) + 2 * (size_t)nch;
  if (h[4] == 2) {
    if (len < pre + 1) return LPCC_E_CORRUPT;
    if (avail < pre + 1) return LPCC_E_CAPACITY;
    H.B = h[pre++];
    if (H.B < 1 || H.B > H.D - 1) return LPCC_E_CORRUPT;
    H.bound = pre + (size_t)H.B * (1 + 5 * 255) + 2 * (size_t)nch;
    H.cnt.assign((size_t)H.B * 255, 0);
    for (int d = 0; d < H.B; d++) {
      if (len < pre + 1) return LPCC_E_CORRUPT;
      if (avail < pre + 1) return LPCC_E_CAPACITY;
      const int mc = h[pre++];
      if (len < pre + 5 * (size_t)mc) return LPCC_E_CORRUPT;
      if (avail < pre + 5 * (size_t)mc) return LPCC_E_CAPACITY;
      int last = 0;
      int64_t sum = 0;
      for (int k = 0; k < mc; k++, pre += 5) {
        const int code = h[pre];
        const uint32_t v = rd32(h + pre + 1);
        if (code <= last || v == 0) return LPCC_E_CORRUPT;
        H.cnt[(size_t)d * 255 + code - 1] = v;
        sum += v;
        last = code;
      }
      if (sum != H.N[d]) return LPCC_E_CORRUPT;
    }
  }
  H.pre = pre;
  H.hdr = pre + 2 * (size_t)nch;
  if (len < H.hdr) return LPCC_E_CORRUPT;
  if (!need_lengths) return LPCC_OK;
  if (avail < H.hdr) return LPCC_E_CAPACITY;
  H.len.resize(nch);
  size_t tot = 0;
  for (int64_t k = 0; k < nch; k++) {
    H.len[k] = (uint32_t)h[pre + 2 * k] | ((uint32_t)h[pre + 2 * k + 1] << 8);
    tot += H.len[k];
  }
  H.total = H.hdr + tot;
  if (H.total != len) return LPCC_E_CORRUPT;
  return LPCC_OK;
}

// Headers of all frames.  Host streams are parsed in place; device streams
// are copied to pinned memory: a prefix that holds the whole header up to
// 4096 chunk lengths for every frame in one round trip, then the rest of any
// longer header in a second one.
constexpr size_t kHdrPrefix = 16 + 4 * kMaxD + 2 * 4096;

int read_headers(lpcc_ctx* c, int nf, const uint8_t* const* bs, const size_t* len, std::vector<Header>& H,
                 std::vector<int>& st) {
  std::vector<size_t> off(nf, 0), got(nf, 0);
  std::vector<bool> dev(nf, false);
  size_t need = 0;
  for (int f = 0; f < nf; f++) {
    st[f] = LPCC_OK;
    if (!bs[f]) {
      st[f] = LPCC_E_INVAL;
      continue;
    }
    dev[f] = is_device_ptr(bs[f]);
    if (!dev[f]) {
      st[f] = parse_header(bs[f], len[f], len[f], H[f], true);
      continue;
    }
    off[f] = need;
    got[f] = std::min(len[f], kHdrPrefix);
    need += align_up(got[f], 64);
  }
  if (need == 0) return LPCC_OK;
  int s = reserve_pinned(c, need);
  if (s) return s;
  for (int f = 0; f < nf; f++)
    if (dev[f] && got[f]) HIPC(hipMemcpyAsync(c->pinned + off[f], bs[f], got[f], hipMemcpyDeviceToHost, c->stream));
  HIPC(stream_wait(c, c->stream));
  std::vector<int> more;
  std::vector<size_t> want(nf, 0);
  size_t need2 = 0;
  for (int f = 0; f < nf; f++) {
    if (!dev[f]) continue;
    st[f] = parse_header(c->pinned + off[f], got[f], len[f], H[f], true);
    if (st[f] == LPCC_E_CAPACITY) {  // longer than the prefix: fetch the whole header
      st[f] = parse_header(c->pinned + off[f], got[f], len[f], H[f], false);
      if (st[f] == LPCC_OK || st[f] == LPCC_E_CAPACITY) {
        // the header's length, or (base tables beyond the prefix) a bound
        want[f] = std::min(len[f], st[f] == LPCC_OK ? H[f].hdr : H[f].bound);
        st[f] = LPCC_OK;
        more.push_back(f);
        need2 += align_up(want[f], 64);
      }
    }
  }
  if (more.empty()) return LPCC_OK;
  // the first round's bytes are parsed; the buffer is reused
  s = reserve_pinned(c, need2);
  if (s) return s;
  size_t o = 0;
  for (int f : more) {
    off[f] = o;
    HIPC(hipMemcpyAsync(c->pinned + o, bs[f], want[f], hipMemcpyDeviceToHost, c->stream));
    o += align_up(want[f], 64);
  }
  HIPC(stream_wait(c, c->stream));
  for (int f : more) {
    st[f] = parse_header(c->pinned + off[f], want[f], len[f], H[f], true);
    if (st[f] == LPCC_E_CAPACITY) st[f] = LPCC_E_CORRUPT;  // the bound held the whole header
  }
  return LPCC_OK;
}

// Decode workspace: per depth keys, codes and first-child rows of all
// frames, the payloads, the CDF rows of the largest depth, error words,
// chunk child counts, staged coordinates, and the model buffers.
struct DecBufs {
  uint8_t* payload = nullptr;
  uint16_t* cdf16 = nullptr;
  uint32_t *err = nullptr, *csum = nullptr;
  int32_t* xyz_stage = nullptr;
};

void carve_decode(Arena& A, const lpcc_model* m, const Frames& fr, size_t paybytes, size_t maxch, bool host_out,
                  int nb, Levels& lv, ModelBufs& B, DecBufs& o) {
  const int D = m->D;
  int64_t maxN = 0;
  for (int d = 0; d <= D; d++) maxN = std::max(maxN, fr.tot[d]);
  std::vector<bool> wanted(D, true);
  for (int d = 0; d < nb && d < D; d++) wanted[d] = false;
  for (int d = 0; d <= D; d++) {
    lv.key[d] = A.take<uint64_t>(fr.tot[d]);
    lv.code[d] = A.take<uint8_t>(align_up(fr.tot[d], 4) + 4);
    lv.cstart[d] = A.take<int32_t>(fr.tot[d] + 1);
  }
  o.payload = A.take<uint8_t>(paybytes);
  o.cdf16 = A.take<uint16_t>((size_t)maxN * 256);
  o.err = A.take<uint32_t>(4);
  o.csum = A.take<uint32_t>(maxch + 1);
  if (host_out) o.xyz_stage = A.take<int32_t>((size_t)fr.tot[D] * 3);
  carve_model(A, m, fr, D - 1, wanted, B, nb);
}

// Arenas a decode of one stream needs, from its depth counts (`N`, D + 1
// entries), base depth and chunk size.  A chunk's payload is at most two
// bytes per symbol (every renormalisation emits at most two) and the flush.
void decode_workspace(const lpcc_model* m, const int64_t* N, int nb, int cl, size_t out[3]) {
  const int D = m->D;
  Frames fr;
  fr.nf = 1;
  fr.tot.assign(N, N + D + 1);
  fr.N.assign(1, fr.tot);
  fr.off.assign(1, std::vector<int64_t>(D + 1, 0));
  size_t maxch = 0, nch = 0, pay = 0;
  for (int d = 0; d < D; d++) {
    maxch = std::max<size_t>(maxch, (size_t)nchunks_of(N[d], cl));
    nch += (size_t)nchunks_of(N[d], cl);
    pay += 2 * (size_t)N[d];
  }
  pay += 8 * nch;
  Levels lv;
  ModelBufs B;
  DecBufs db;
  Arena a;
  carve_decode(a, m, fr, align_up(pay, 16), maxch, true, nb, lv, B, db);
  out[0] = 0;
  out[1] = a.off + 4096;
  out[2] = desc_bound(fr, nch);
}

}  // namespace

void lpcc::decode_workspace_bound(const lpcc_model* m, int nf, const int64_t* const* N, const int* cl,
                                  size_t out[3]) {
  const int D = m->D;
  Frames fr;
  fr.nf = nf;
  fr.tot.assign(D + 1, 0);
  fr.N.assign(nf, std::vector<int64_t>(D + 1, 0));
  fr.off.assign(nf, std::vector<int64_t>(D + 1, 0));
  std::vector<size_t> dch(D, 0);
  size_t nch = 0, pay = 0;
  for (int f = 0; f < nf; f++)
    for (int d = 0; d <= D; d++) {
      fr.N[f][d] = N[f][d];
      fr.off[f][d] = fr.tot[d];
      fr.tot[d] += N[f][d];
      if (d < D) {
        const size_t k = (size_t)nchunks_of(N[f][d], cl[f]);
        dch[d] += k;
        nch += k;
        pay += 2 * (size_t)N[f][d] + 8 * k + 16;
      }
    }
  size_t maxch = 0;
  for (int d = 0; d < D; d++) maxch = std::max(maxch, dch[d]);
  Levels lv;
  ModelBufs B;
  DecBufs db;
  Arena a;
  carve_decode(a, m, fr, align_up(pay, 16), maxch, true, 0, lv, B, db);
  out[0] = 0;
  out[1] = a.off + 4096;
  out[2] = desc_bound(fr, nch);
}

void lpcc::ctx_caps(const lpcc_ctx* c, size_t caps[3]) {
  for (int i = 0; i < 3; i++) caps[i] = c->fixed ? 0 : c->cap[i];
}
void lpcc::ctx_set_budget(lpcc_ctx* c, size_t budget) { c->budget = budget; }
void lpcc::ctx_trim(lpcc_ctx* c) {
  if (c->fixed) return;
  (void)hipStreamSynchronize(c->stream);
  for (int i = 0; i < 3; i++) {
    if (c->dev[i]) (void)hipFree(c->dev[i]);
    c->dev[i] = nullptr;
    c->cap[i] = 0;
  }
}

namespace {

int decode_impl(lpcc_ctx* c, const lpcc_model* m, int nf, const uint8_t* const* bs, const size_t* len,
                int32_t* const* xyz_out, const int64_t* cap, int64_t* n_out, int* status) {
  const int D = m->D, C = m->C, k0 = m->k0;
  resolve_tuning(c);
  c->call_kind = 1;
  c->batch_idx = 0;
  hipStream_t st = c->stream;
  std::vector<Header> H(nf);
  std::vector<int> live, hst(nf, LPCC_OK);
  {
    const int s = read_headers(c, nf, bs, len, H, hst);
    if (s) return s;
  }
  for (int f = 0; f < nf; f++) {
    n_out[f] = 0;
    int s = hst[f];
    if (s == LPCC_OK && (H[f].D != D || H[f].n_deep != m->n_deep || H[f].blob != m->blob_id)) s = LPCC_E_MODEL;
    if (s == LPCC_OK) {
      n_out[f] = H[f].N[D];
      if (H[f].N[D] > cap[f]) s = LPCC_E_CAPACITY;
    }
    status[f] = s;
    if (s == LPCC_OK && H[f].N[D] > 0) live.push_back(f);
  }
  // the frames of one call share the base depth; a call whose frames differ
  // decodes them one at a time
  const int nb = live.empty() ? 0 : H[live[0]].B;
  for (int f : live)
    if (H[f].B != nb) {
      for (int g : live) {
        int st1 = LPCC_OK;
        int64_t n1 = 0;
        decode_impl(c, m, 1, &bs[g], &len[g], &xyz_out[g], &cap[g], &n1, &st1);
        status[g] = st1;
        n_out[g] = n1;
      }
      int ret = LPCC_OK;
      for (int g = 0; g < nf; g++)
        if (status[g] != LPCC_OK && ret == LPCC_OK) ret = status[g];
      return ret;
    }
  if (nb > k0) {  // a base depth the model cannot continue from
    for (int f : live) status[f] = LPCC_E_CORRUPT;
    return LPCC_E_CORRUPT;
  }
  Frames fr;
  fr.nf = nf;
  fr.tot.assign(D + 1, 0);
  fr.N.assign(nf, std::vector<int64_t>(D + 1, 0));
  fr.off.assign(nf, std::vector<int64_t>(D + 1, 0));
  for (int f : live)
    for (int d = 0; d <= D; d++) {
      fr.off[f][d] = fr.tot[d];
      fr.N[f][d] = H[f].N[d];
      fr.tot[d] += H[f].N[d];
    }
  if (live.empty()) {
    int ret = LPCC_OK;
    for (int f = 0; f < nf; f++)
      if (status[f] != LPCC_OK && ret == LPCC_OK) ret = status[f];
    return ret;
  }
  // chunks per depth (all frames), payload placement
  std::vector<std::vector<Chunk>> dchunks(D);
  std::vector<size_t> dmaxlen(D, 0);
  size_t paybytes = 0;
  std::vector<size_t> payoff(nf, 0);
  for (int f : live) {
    payoff[f] = paybytes;
    paybytes += align_up(H[f].total - H[f].hdr, 16);
    size_t ci = 0, po = payoff[f];
    const int cl = H[f].cl;
    for (int d = 0; d < D; d++) {
      const int64_t Nfd = H[f].N[d];
      for (int64_t k = 0; k < nchunks_of(Nfd, cl); k++) {
        Chunk ch;
        ch.node0 = fr.off[f][d] + (k << cl);
        ch.count = (int32_t)std::min<int64_t>(1ll << cl, Nfd - (k << cl));
        ch.pad_ = (int32_t)H[f].len[ci];
        ch.scratch = (int64_t)po;
        po += H[f].len[ci];
        dmaxlen[d] = std::max<size_t>(dmaxlen[d], H[f].len[ci]);
        dchunks[d].push_back(ch);
        ci++;
      }
    }
  }
  Levels lv;
  ModelBufs B;
  B.hash_all = c->kmap_mode == 1;
  size_t maxch = 0;
  for (int d = 0; d < D; d++) maxch = std::max(maxch, dchunks[d].size());
  std::vector<bool> xdev(nf, false);
  bool any_host_out = false;
  for (int f : live) {
    xdev[f] = is_device_ptr(xyz_out[f]);
    if (!xdev[f]) any_host_out = true;
  }
  DecBufs db;
  Arena meas;
  carve_decode(meas, m, fr, paybytes, maxch, any_host_out, nb, lv, B, db);
  int s = reserve(c, 1, meas.off + 4096);
  if (s) return s;
  Arena A;
  A.base = c->dev[1];
  A.cap = c->cap[1];
  carve_decode(A, m, fr, paybytes, maxch, any_host_out, nb, lv, B, db);
  uint8_t* payload = db.payload;
  uint16_t* cdf16 = db.cdf16;
  uint32_t *err = db.err, *csum = db.csum;
  int32_t* xyz_stage = db.xyz_stage;
  size_t desc_off = 0;

  // payloads and roots: one device-resident stream is read in place (its
  // chunk offsets already start at 0), others are gathered into one buffer
  if (live.size() == 1 && is_device_ptr(bs[live[0]])) {
    payload = const_cast<uint8_t*>(bs[live[0]]) + H[live[0]].hdr;
  } else {
    for (int f : live) {
      const size_t pl = H[f].total - H[f].hdr;
      if (!pl) continue;
      HIPC(hipMemcpyAsync(payload + payoff[f], bs[f] + H[f].hdr, pl,
                          is_device_ptr(bs[f]) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    }
  }
  // V_0: one root per live frame; its key is the frame's position tag
  HIPC(launch_iota_u64(lv.key[0], (int64_t)live.size(), st));
  HIPC(launch_fill_u32(err, 4, 0, st));

  Batch b;
  b.ctx = c;
  {
    // F_B = 0: the first modelled depth has no coarser context
    int8_t* f0 = B.F[nb];
    const int64_t bytes = fr.tot[nb] * C;
    b.launch("fill", 0, [=](const uint8_t*) { return launch_fill_u32((uint32_t*)f0, (bytes + 3) / 4, 0, st); });
  }
  size_t brow_off = 0;  // descriptor offset of the base rows [live frame][depth][256]
  if (nb > 0) {
    // 16-bit CDF rows of the base depths (entry 255 is not a boundary: 0)
    std::vector<uint16_t> rows(live.size() * nb * 256, 0);
    for (size_t i = 0; i < live.size(); i++)
      for (int d = 0; d < nb; d++) {
        int32_t cdf[256];
        base_cdf(H[live[i]].cnt.data() + (size_t)d * 255, cdf);
        uint16_t* r = rows.data() + (i * nb + d) * 256;
        for (int k = 0; k < 255; k++) r[k] = (uint16_t)cdf[k];
      }
    brow_off = b.add(rows);
  }
  plan_hash_clear(b, B, st);
  if (nb == 0 && B.kmap[0]) plan_kmaps(b, lv, fr, B, {0}, st);
  // Depth d's chain is predictor -> coder -> expansion -> upsampling of
  // depth d+1.  The ResBlock of depth d+1 needs only F_d and the neighbour
  // table of depth d, and the neighbour table of depth d+1 only the
  // expansion, so both run on a second stream beside the chain.
  c->sync_used = 0;
  bool two = c->time_family.empty() && !c->graphs && !c->fixed;
  if (two && !c->side && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    c->side = nullptr;
  }
  two = two && c->side;
  // Depths with few nodes stay on one stream: their kernels are short, and
  // the event records and waits of the split would cost the host more than
  // the overlap gains.  The split starts at the first depth of kSplitRows
  // nodes (node counts only grow with depth) and lasts to the end.
  constexpr int64_t kSplitRows = 16384;
  int dsplit = D;
  for (int d = 0; d < D; d++)
    if (fr.tot[d] >= kSplitRows) {
      dsplit = d;
      break;
    }
  bool two_now = false;  // this iteration runs work on the side stream
  hipStream_t sd = st;
  bool ok_ev = true;
  // record an event on `s` now (null while one stream is used)
  auto mark = [&](hipStream_t s) -> hipEvent_t {
    if (!two_now) return nullptr;
    hipEvent_t e = sync_event(c);
    if (!e) {
      ok_ev = false;
      return nullptr;
    }
    plan_record(b, e, s);
    return e;
  };
  auto wait = [&](hipStream_t s, hipEvent_t e) {  // an event from an earlier split iteration still counts
    if (e) plan_wait(b, s, e);
  };
  auto join = [&](hipStream_t from, hipStream_t to) {
    wait(to, mark(from));
    return true;
  };
  hipEvent_t kmap_k0 = nullptr;
  for (int d = 0; d < D; d++) {
    two_now = two && d >= dsplit;
    sd = two_now ? c->side : st;
    const int t = d + 1;  // the shallow depth whose features this iteration prepares
    if (d > k0) {
      if (d == k0 + 1) wait(st, kmap_k0);  // the neighbour table of k0
      plan_deep(b, m, lv, fr, B, {d}, st);
    }
    hipEvent_t resblock = nullptr;
    const bool modelled = d >= nb;  // base depths carry no features
    // the ResBlock of depth t reads F_d (now), or without cross-scale
    // propagation the codes X_d (after the coder below)
    if (t <= k0 && modelled && m->xfp) {
      join(st, sd);  // F_d
      plan_shallow_convs(b, m, lv, fr, B, t, sd);
      resblock = mark(sd);
    }
    if (modelled) {
      PredSeg p;
      memset(&p, 0, sizeof(p));
      p.F = features_of(m, B, d);
      p.fc1 = dlayer(m, d, m->first[d + 1] - m->first[d] - 2);
      p.fc2 = dlayer(m, d, m->first[d + 1] - m->first[d] - 1);
      p.rows = (int)fr.tot[d];
      p.cdf16 = cdf16;
      plan_predict(b, m, {p}, 1, st);
    } else {
      // the CDF row of every node of this base depth is its frame's table
      const uint64_t* keys = lv.key[d];
      const int64_t nd_ = fr.tot[d];
      const int dd = d, nb_ = nb, nl = (int)live.size();
      const size_t ro = brow_off;
      b.launch("base", nd_, [=](const uint8_t* base) {
        return launch_base_rows(keys, nd_, dd, nb_, nl, (const uint16_t*)(base + ro), cdf16, st);
      });
    }
    const size_t co = b.add(dchunks[d]);
    const int nch = (int)dchunks[d].size();
    {
      const size_t ml = dmaxlen[d];
      uint8_t* codes = lv.code[d];
      uint32_t* cs = csum;
      b.launch("rc_decode", fr.tot[d], [=](const uint8_t* base) {
        return launch_rc_decode_sized((const Chunk*)(base + co), nch, payload, cdf16, codes, cs, err + 0, ml, st);
      });
    }
    if (t <= k0 && modelled && !m->xfp) {
      join(st, sd);  // X_d decoded
      plan_shallow_convs(b, m, lv, fr, B, t, sd);
      resblock = mark(sd);
    }
    {
      // children of depth d from the chunks' child counts; when depth d+1
      // convolves, its hash table is filled on the way
      const uint64_t* pk = lv.key[d];
      const uint8_t* codes = lv.code[d];
      const int64_t np = fr.tot[d], nc = fr.tot[d + 1];
      uint64_t* ck = lv.key[d + 1];
      int32_t* cst = lv.cstart[d];
      uint32_t* e1 = err + 1;
      uint32_t* cs = csum;
      const bool hashed = d + 1 <= k0 && d + 1 >= nb && B.kmap[d + 1] && !B.tree[d + 1];
      uint64_t* tk = hashed ? B.hkeys[d + 1] : nullptr;
      const uint64_t hm = hashed ? B.hmask[d + 1] : 0;
      b.launch("expand", np, [=](const uint8_t* base) {
        return launch_expand_chunks((const Chunk*)(base + co), nch, pk, codes, np, cs, ck, cst, nc, tk, hm, e1,
                                    st);
      });
    }
    if (t <= k0 && t >= nb && B.kmap[t]) {
      join(st, sd);  // the expansion: hash table or first-child rows of depth d
      if (B.tree[t])
        plan_kmap_tree(b, lv, fr, B, t, sd);
      else
        plan_kmap_only(b, lv, fr, B, t, sd);
      if (t == k0) kmap_k0 = mark(sd);
    }
    if (t <= k0 && modelled) {
      wait(st, resblock);  // the ResBlock output (not the neighbour table)
      plan_shallow_up(b, m, lv, fr, B, t, st);
    }
    // From the first large depth on the GPU is the bottleneck: submit what
    // is planned, so that planning the remaining depths overlaps its work
    // (every later launch uses descriptors added after this point)
    if (d == dsplit && d + 1 < D && d + 1 >= nb && !c->graphs) {
      if (!ok_ev) {
        c->err = "event creation failed";
        return LPCC_E_DEVICE;
      }
      s = run_batch(c, b, &desc_off);
      if (s) return s;
    }
  }
  if (two && dsplit < D) {  // the main stream waits for the side stream's last work
    two_now = true;
    join(c->side, st);
  }
  if (!ok_ev) {
    c->err = "event creation failed";
    return LPCC_E_DEVICE;
  }
  s = run_batch(c, b, &desc_off);
  if (s) return s;
  // coordinates, enqueued before the error words are read (a corrupt frame
  // only writes within its own output; its status then reports the error)
  for (int f : live) {
    const uint64_t* keys = lv.key[D] + fr.off[f][D];
    int32_t* dst = xdev[f] ? xyz_out[f] : xyz_stage + 3 * fr.off[f][D];
    HIPC(launch_keys_to_xyz(keys, fr.N[f][D], D, dst, st));
    if (!xdev[f])
      HIPC(hipMemcpyAsync(xyz_out[f], dst, (size_t)fr.N[f][D] * 12, hipMemcpyDeviceToHost, st));
  }
  s = reserve_pinned(c, desc_off + 256);
  if (s) return s;
  uint32_t* herr = (uint32_t*)(c->pinned + c->pinned_cap - 256);
  HIPC(hipMemcpyAsync(herr, err, 16, hipMemcpyDeviceToHost, st));
  HIPC(stream_wait(c, st));
  if (herr[0] | herr[1]) {
    // a corrupt frame misaligns the shared arrays: report per frame by
    // decoding the frames one at a time
    if (live.size() == 1) {
      status[live[0]] = LPCC_E_CORRUPT;
      return LPCC_E_CORRUPT;
    }
    for (int f : live) {
      int st1 = LPCC_OK;
      int64_t n1 = 0;
      decode_impl(c, m, 1, &bs[f], &len[f], &xyz_out[f], &cap[f], &n1, &st1);
      status[f] = st1;
    }
    int ret = LPCC_OK;
    for (int f = 0; f < nf; f++)
      if (status[f] != LPCC_OK && ret == LPCC_OK) ret = status[f];
    return ret;
  }
  int ret = LPCC_OK;
  for (int f = 0; f < nf; f++)
    if (status[f] != LPCC_OK && ret == LPCC_OK) ret = status[f];
  return ret;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int lpcc_model_load(const void* blob, size_t len, int device, lpcc_model** out) {
  if (!blob || !out) return LPCC_E_INVAL;
  *out = nullptr;
  std::unique_ptr<lpcc_model> m(new lpcc_model());
  m->device = device;
  int s = parse_blob((const uint8_t*)blob, len, m.get());
  if (s) return s;
  if (hipSetDevice(device) != hipSuccess) return LPCC_E_DEVICE;
  // one device block: per layer packed W, raw W, bias, zc; then the table
  std::vector<LayerImage> im;
  size_t bytes = 0;
  for (size_t i = 0; i < m->host.size(); i++) {
    const HostLayer& L = m->host[i];
    im.push_back(build_image(L));
    const bool own = L.owner == (int)i;  // shared weights are placed once, with their owner
    bytes += (own ? align_up(im.back().packed.size(), 256) + align_up(L.W.size(), 256) : 0) +
             align_up(im.back().bias.size() * 4, 256) + align_up(im.back().zc.size() * 4, 256);
  }
  bytes += 1024 + align_up(m->host.size() * sizeof(LayerDev), 256);
  std::vector<uint8_t> host(bytes, 0);
  if (hipMalloc(&m->d_mem, bytes) != hipSuccess) return LPCC_E_NOMEM;
  uint8_t* dbase = (uint8_t*)m->d_mem;
  size_t off = 0;
  auto put = [&](const void* src, size_t n) -> uint8_t* {
    uint8_t* d = dbase + off;
    if (n) memcpy(host.data() + off, src, n);
    off += align_up(n, 256);
    return d;
  };
  std::vector<LayerDev> ld(m->host.size());
  for (size_t i = 0; i < m->host.size(); i++) {
    const HostLayer& L = m->host[i];
    LayerDev& D = ld[i];
    memset(&D, 0, sizeof(D));
    if (L.owner == (int)i) {
      D.Wp = (const int8_t*)put(im[i].packed.data(), im[i].packed.size());
      D.Wr = (const int8_t*)put(L.W.data(), L.W.size());
    } else {
      D.Wp = ld[L.owner].Wp;
      D.Wr = ld[L.owner].Wr;
    }
    D.bias = (const int32_t*)put(im[i].bias.data(), im[i].bias.size() * 4);
    D.zc = im[i].zc.empty() ? nullptr : (const int32_t*)put(im[i].zc.data(), im[i].zc.size() * 4);
    const RqBounds rq = requant_bounds(L.m_pos, L.m_neg, L.r, L.z_out);
    D.m_pos = rq.m_pos;
    D.m_neg = rq.m_neg;
    D.a_lo = rq.a_lo;
    D.a_hi = rq.a_hi;
    D.r = L.r;
    D.z_out = L.z_out;
    D.taps = L.taps;
    D.cin = L.cin;
    D.cout = L.cout;
    D.ksteps = im[i].ksteps;
    D.npad = im[i].npad;
    D.rnd = L.r > 0 ? (1ll << (L.r - 1)) : 0;
    D.rq24 = requant_fits24(D.m_pos, D.m_neg, D.a_lo, D.a_hi, D.rnd) ? 1 : 0;
  }
  int32_t lut[256];
  softmax_table(lut);
  m->d_lut = (int32_t*)put(lut, sizeof(lut));
  m->d_layers = (LayerDev*)put(ld.data(), ld.size() * sizeof(LayerDev));
  m->h_layers = ld;
  if (hipMemcpy(m->d_mem, host.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(m->d_mem);
    return LPCC_E_DEVICE;
  }
  *out = m.release();
  return LPCC_OK;
}

void lpcc_model_free(lpcc_model* m) {
  if (!m) return;
  if (m->d_mem) (void)hipFree(m->d_mem);
  delete m;
}

int lpcc_model_info(const lpcc_model* m, int* C, int* D, int* n_deep, uint32_t* blob_id) {
  if (!m) return LPCC_E_INVAL;
  if (C) *C = m->C;
  if (D) *D = m->D;
  if (n_deep) *n_deep = m->n_deep;
  if (blob_id) *blob_id = m->blob_id;
  return LPCC_OK;
}

int lpcc_ctx_create(int device, void* hip_stream, size_t hbm_budget, lpcc_ctx** out) {
  if (!out) return LPCC_E_INVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return LPCC_E_DEVICE;
  lpcc_ctx* c = new lpcc_ctx();
  c->device = device;
  c->budget = hbm_budget;
  // companion of the allocation-free entry point: the device address of the
  // library's static block (looked up once per device, with `device` current)
  // and a pageable host staging buffer of fixed size
  c->noalloc = new lpcc_ctx();
  c->noalloc->device = device;
  c->noalloc->fixed = true;
  if (lpcc::scratch_setup(device, &c->noalloc->fixed_base, &c->noalloc->fixed_cap, &c->noalloc->fixed_why) ==
      LPCC_OK) {
    c->noalloc->hostbuf.reset(new uint8_t[lpcc::kNoallocHost]);
    c->noalloc->pinned = c->noalloc->hostbuf.get();
    c->noalloc->pinned_cap = lpcc::kNoallocHost;
  }
  c->stream = (hipStream_t)hip_stream;
  if (!c->stream) {
    if (hipStreamCreate(&c->own_stream) != hipSuccess) {
      delete c;
      return LPCC_E_DEVICE;
    }
    c->stream = c->own_stream;
  }
  c->noalloc->stream = c->stream;
  *out = c;
  return LPCC_OK;
}

void lpcc_ctx_free(lpcc_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->noalloc) lpcc_ctx_free(c->noalloc);
  for (int i = 0; i < 3 && !c->fixed; i++)
    if (c->dev[i]) (void)hipFree(c->dev[i]);
  if (c->pinned && !c->fixed) (void)hipHostFree(c->pinned);
  for (auto& e : c->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.z);
  }
  for (auto e : c->ev_free) (void)hipEventDestroy(e);
  for (auto& kv : c->gexec) (void)hipGraphExecDestroy(kv.second);
  for (auto e : c->sync_ev) (void)hipEventDestroy(e);
  if (c->poll_ev) (void)hipEventDestroy(c->poll_ev);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

const char* lpcc_last_error(const lpcc_ctx* c) { return c ? c->err.c_str() : "null context"; }

int lpcc_ctx_workspace(const lpcc_ctx* c, size_t* held, size_t* peak) {
  if (!c) return LPCC_E_INVAL;
  if (held) *held = held_bytes(c);
  if (peak) *peak = c->peak;
  return LPCC_OK;
}

int lpcc_peek_header(const uint8_t* bs, size_t len, int* D, int64_t* n_points, size_t* max_workspace) {
  if (!bs) return LPCC_E_INVAL;
  if (len < 16 || bs[0] != 'L' || bs[1] != 'P' || bs[2] != 'C' || bs[3] != '1' || (bs[4] != 1 && bs[4] != 2))
    return LPCC_E_CORRUPT;
  if (bs[5] < 1 || bs[5] > kMaxD) return LPCC_E_CORRUPT;
  if (D) *D = bs[5];
  if (n_points) *n_points = rd32(bs + 12);
  if (max_workspace) {
    *max_workspace = 0;
    Header H;  // `len` bytes of a stream of unknown length
    const int st = parse_header(bs, len, (size_t)1 << 62, H, false);
    if (st == LPCC_OK && H.n_deep <= H.D - 1) {
      // the larger of the two schedules at the widest model
      size_t best = 0;
      for (int xfp = 0; xfp <= 1; xfp++) {
        lpcc_model shape;
        shape.C = 64;
        shape.D = H.D;
        shape.n_deep = H.n_deep;
        shape.k0 = H.D - H.n_deep - 1;
        shape.xfp = xfp;
        size_t w[3];
        decode_workspace(&shape, H.N.data(), H.B, H.cl, w);
        best = std::max(best, w[0] + w[1] + w[2]);
      }
      *max_workspace = best;
    } else if (st != LPCC_OK && st != LPCC_E_CAPACITY) {
      return st;
    }
  }
  return LPCC_OK;
}

int lpcc_encode_batch(lpcc_ctx* c, const lpcc_model* m, int nf, const int32_t* const* xyz, const int64_t* n,
                      int chunk_log2, uint8_t* const* out, const size_t* cap, size_t* out_len, int* status) {
  if (!c || !m || nf <= 0 || !xyz || !n || !out || !cap || !out_len || !status) return LPCC_E_INVAL;
  if (chunk_log2 < 4 || chunk_log2 > 14) return LPCC_E_INVAL;
  for (int f = 0; f < nf; f++)
    if (n[f] < 0 || (n[f] > 0 && !xyz[f]) || n[f] > (1ll << 30)) return LPCC_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return LPCC_E_DEVICE;
  c->err.clear();
  OutSpec os{out, cap, out_len};
  return encode_impl(c, m, nf, xyz, n, chunk_log2, os, status, -1, nullptr, 0, nullptr);
}

int lpcc_encode_frame(lpcc_ctx* c, const lpcc_model* m, const int32_t* xyz, int64_t n, int chunk_log2,
                      uint8_t* out, size_t cap, size_t* out_len) {
  if (!out_len) return LPCC_E_INVAL;
  int st = 0;
  return lpcc_encode_batch(c, m, 1, &xyz, &n, chunk_log2, &out, &cap, out_len, &st);
}

int lpcc_encode_frame_noalloc(lpcc_ctx* c, const lpcc_model* m, const int32_t* xyz, int64_t n, int chunk_log2,
                              uint8_t* out, size_t cap, size_t* out_len) {
  if (!c || !m || !out || !out_len || n < 0 || (n > 0 && !xyz) || n > (1ll << 30)) return LPCC_E_INVAL;
  if (chunk_log2 < 4 || chunk_log2 > 14) return LPCC_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return LPCC_E_DEVICE;
  c->err.clear();
  lpcc_ctx* z = c->noalloc;
  if (!z || !z->fixed_base) {
    c->err = z ? z->fixed_why : std::string("context without an allocation-free companion");
    return LPCC_E_DEVICE;
  }
  // every call on the device carves the same block: one call at a time, held
  // until the call's work has finished (the call is synchronous)
  std::lock_guard<std::mutex> g(lpcc::scratch_mutex(c->device));
  z->stream = c->stream;
  z->base = c->base;
  z->tiling = c->tiling;
  z->err.clear();
  int st = 0;
  OutSpec os{&out, &cap, out_len};
  const int s = encode_impl(z, m, 1, &xyz, &n, chunk_log2, os, &st, -1, nullptr, 0, nullptr);
  if (s) c->err = z->err;
  return s;
}

int lpcc_level_probs(lpcc_ctx* c, const lpcc_model* m, const int32_t* xyz, int64_t n, int level, int32_t* cdf_out,
                     int64_t cap, int64_t* n_nodes) {
  if (!c || !m || !n_nodes || n < 0 || (n > 0 && !xyz)) return LPCC_E_INVAL;
  if (level < 0 || level >= m->D) return LPCC_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return LPCC_E_DEVICE;
  c->err.clear();
  int st = 0;
  size_t dummy = 0;
  OutSpec os{nullptr, &dummy, &dummy};
  *n_nodes = 0;
  return encode_impl(c, m, 1, &xyz, &n, 10, os, &st, level, cdf_out, cap, n_nodes);
}

int lpcc_decode_batch(lpcc_ctx* c, const lpcc_model* m, int nf, const uint8_t* const* bs, const size_t* len,
                      int32_t* const* xyz_out, const int64_t* cap, int64_t* n_out, int* status) {
  if (!c || !m || nf <= 0 || !bs || !len || !xyz_out || !cap || !n_out || !status) return LPCC_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return LPCC_E_DEVICE;
  c->err.clear();
  return decode_impl(c, m, nf, bs, len, xyz_out, cap, n_out, status);
}

int lpcc_decode_frame(lpcc_ctx* c, const lpcc_model* m, const uint8_t* bs, size_t len, int32_t* xyz_out,
                      int64_t cap, int64_t* n_out) {
  if (!n_out) return LPCC_E_INVAL;
  int st = 0;
  return lpcc_decode_batch(c, m, 1, &bs, &len, &xyz_out, &cap, n_out, &st);
}

int lpcc_timing_enable(lpcc_ctx* c, const char* name) {
  if (!c) return LPCC_E_INVAL;
  c->time_family = name ? name : "";
  c->ev_used = 0;
  c->time_units = 0;
  return LPCC_OK;
}

int lpcc_timing_read(lpcc_ctx* c, int64_t* launches, double* total_ms, int64_t* units) {
  if (!c) return LPCC_E_INVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LPCC_E_DEVICE;
  double tot = 0;
  for (size_t i = 0; i < c->ev_used; i++) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev[i].first, c->ev[i].second) != hipSuccess) return LPCC_E_DEVICE;
    tot += ms;
  }
  if (launches) *launches = (int64_t)c->ev_used;
  if (total_ms) *total_ms = tot;
  if (units) *units = c->time_units;
  c->ev_used = 0;
  c->time_units = 0;
  return LPCC_OK;
}

int lpcc_ctx_set_graphs(lpcc_ctx* c, int on) {
  if (!c) return LPCC_E_INVAL;
  c->graphs = on ? 1 : 0;
  return LPCC_OK;
}

int lpcc_ctx_graph_stats(lpcc_ctx* c, int64_t* instantiated, int64_t* updated) {
  if (!c) return LPCC_E_INVAL;
  if (instantiated) *instantiated = c->graph_inst;
  if (updated) *updated = c->graph_upd;
  return LPCC_OK;
}

int lpcc_ctx_set_tiling(lpcc_ctx* c, int rb) {
  if (!c || !(rb == 0 || rb == 1 || rb == 2 || rb == 4 || rb == 11 || rb == 12 || rb == 14)) return LPCC_E_INVAL;
  c->tiling = rb;
  return LPCC_OK;
}

int lpcc_ctx_set_kmap_mode(lpcc_ctx* c, int mode) {
  if (!c || (mode != 0 && mode != 1)) return LPCC_E_INVAL;
  c->kmap_mode = mode;
  return LPCC_OK;
}

int lpcc_ctx_set_base_depth(lpcc_ctx* c, int base) {
  if (!c || base < 0 || base >= kMaxD) return LPCC_E_INVAL;
  c->base = base;
  return LPCC_OK;
}

int lpcc_ctx_tuning(lpcc_ctx* c, int32_t* out, int cap, int* n) {
  if (!c || !n) return LPCC_E_INVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LPCC_E_DEVICE;
  resolve_tuning(c);
  int k = 0;
  for (auto& kv : c->tune) {
    if (out && k < cap) {
      for (int i = 0; i < 5; i++) out[6 * k + i] = kv.first[i];
      out[6 * k + 5] = kv.second.best;
    }
    k++;
  }
  *n = k;
  return k > cap && out ? LPCC_E_CAPACITY : LPCC_OK;
}

int lpcc_ctx_set_tuning(lpcc_ctx* c, const int32_t* rows, int n) {
  if (!c || n < 0 || (n > 0 && !rows)) return LPCC_E_INVAL;
  // every row is checked before any is applied
  for (int k = 0; k < n; k++) {
    const int32_t* r = rows + 6 * k;
    if (r[0] != 0 && r[0] != 1) return LPCC_E_INVAL;
    if (r[2] <= 0 || r[3] <= 0 || r[4] < 0 || r[4] > 62) return LPCC_E_INVAL;
    if (r[5] == 0) continue;
    bool known = false;
    for (const Variant& v : variants(r[0] == 1, r[1])) known = known || v.code == r[5];
    if (!known) return LPCC_E_INVAL;
  }
  for (int k = 0; k < n; k++) {
    const int32_t* r = rows + 6 * k;
    if (r[5] != 0) c->tune[{r[0], r[1], r[2], r[3], r[4]}].best = r[5];
  }
  return LPCC_OK;
}

// Exponent table of the integer softmax as the library builds it (host only).
int lpcc_softmax_table(int32_t* out) {
  if (!out) return LPCC_E_INVAL;
  softmax_table(out);
  return LPCC_OK;
}

// Accumulator bounds of one requantisation as the kernels use them (host only).
int lpcc_requant_bounds(int32_t m_pos, int32_t m_neg, int r, int z_out, int32_t* out) {
  if (!out || m_pos < 0 || m_neg < 0 || r < 0 || r > 62 || z_out < -128 || z_out > 127) return LPCC_E_INVAL;
  const RqBounds B = requant_bounds(m_pos, m_neg, r, z_out);
  out[0] = B.m_pos;
  out[1] = B.m_neg;
  out[2] = B.a_lo;
  out[3] = B.a_hi;
  out[4] = requant_fits24(B.m_pos, B.m_neg, B.a_lo, B.a_hi, r > 0 ? (1ll << (r - 1)) : 0) ? 1 : 0;
  return LPCC_OK;
}

}  // extern "C"
