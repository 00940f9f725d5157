// Seeded random-init weight blobs (host code).  The per-depth layer list is
// the model of Sec. S2 with the schedule of Sec. 3.1-3.2 (re-densified deep
// depths from k0 = D - n_deep - 1 on); every layer carries int8 weights, an
// int32 bias and the multiply-shift requantisation of Eq. 12-14.  Values come
// from SplitMix64 (Steele, Lea & Flood 2014) in counter form, so a blob is a
// pure function of its arguments.  Integer arithmetic only: the requantisation
// multiplier floor(2^24 / (73.6 sqrt(K))) of a layer with fan-in K is the
// largest m with m^2 * 736^2 * K <= (10 * 2^24)^2.
#include <cstring>
#include <vector>

#include "lpcc_internal.h"

namespace {

constexpr uint32_t kBlobMagic = 0x5743504Cu;  // "LPCW"
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

uint64_t splitmix(uint64_t seed, uint64_t k) {  // output k >= 1
  uint64_t z = seed + k * kGamma;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// largest m >= 0 with m^2 * 736^2 * K <= (167772160)^2 (all below 2^63)
int64_t unit_gain_multiplier(int64_t K) {
  const unsigned __int128 T = (unsigned __int128)167772160ull * 167772160ull;
  int64_t lo = 0, hi = 1ll << 25;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    const unsigned __int128 v = (unsigned __int128)mid * (unsigned __int128)mid * 541696u * (unsigned __int128)K;
    if (v <= T) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct Rec {
  int kind, depth, j, taps, cin, cout;
};

// Layers in blob order (the same list the loader validates)
std::vector<Rec> plan(int C, int D, int n_deep, bool xfp) {
  const int k0 = D - n_deep - 1;
  std::vector<Rec> v;
  for (int d = 0; d < D; d++) {
    if (d >= 1 && d <= k0) {
      if (!xfp) v.push_back({lpcc::K_EMB, d, d - 1, 1, 8, C});
      v.push_back({lpcc::K_CONV1, d, 0, 27, C, C});
      v.push_back({lpcc::K_CONV2, d, 0, 27, C, C});
      v.push_back({lpcc::K_UP, d, d - 1, 1, C + 8, 8 * C});
    } else if (d > k0) {
      v.push_back({lpcc::K_EMB, d, d - 1, 1, 8, C});
      for (int j = d - 1; j > k0; j--) v.push_back({lpcc::K_DOWN, d, j, 8, C, C});
      if (xfp) {
        v.push_back({lpcc::K_CONV1, d, k0, 27, 2 * C, C});
        v.push_back({lpcc::K_CONV2, d, k0, 27, C, C});
        v.push_back({lpcc::K_SKIP, d, k0, 1, 2 * C, C});
      } else {
        v.push_back({lpcc::K_CONV1, d, k0, 27, C, C});
        v.push_back({lpcc::K_CONV2, d, k0, 27, C, C});
      }
      for (int j = k0; j < d; j++) v.push_back({lpcc::K_UP, d, j, 1, C + 8, 8 * C});
    }
    v.push_back({lpcc::K_FC1, d, d, 1, C, C});
    v.push_back({lpcc::K_FC2, d, d, 1, C, lpcc::kNSym});
  }
  return v;
}

// Level-aware parameter sharing: the layer whose weights each layer uses.
// One role per kind for the shallow depths (d <= k0) and one for the deep
// depths, one per predictor layer for all depths; the first layer of a role
// in blob order owns the weights.
std::vector<int> owners(const std::vector<Rec>& layers, int k0) {
  std::vector<int> own(layers.size());
  std::vector<std::pair<int, int>> roles;  // (role key, owner)
  for (size_t i = 0; i < layers.size(); i++) {
    const Rec& L = layers[i];
    const int key = (L.kind == lpcc::K_FC1 || L.kind == lpcc::K_FC2) ? 2 * L.kind : 2 * L.kind + (L.depth > k0 ? 1 : 0);
    int o = (int)i;
    for (auto& r : roles)
      if (r.first == key) o = r.second;
    if (o == (int)i) roles.push_back({key, (int)i});
    own[i] = o;
  }
  return own;
}

void put32(std::vector<uint8_t>& b, uint32_t v) {
  for (int k = 0; k < 4; k++) b.push_back((uint8_t)(v >> (8 * k)));
}

}  // namespace

extern "C" int lpcc_make_weights(uint64_t seed, int C, int D, int n_deep, int flags, void* blob, size_t cap,
                                 size_t* len) {
  if (!len || !(C == 16 || C == 32 || C == 64) || D < 1 || D > lpcc::kMaxD || n_deep < 0 || n_deep > D - 1 ||
      (flags & ~(LPCC_W_NO_XFP | LPCC_W_ZERO_POINTS | LPCC_W_SHARED)))
    return LPCC_E_INVAL;
  const bool xfp = !(flags & LPCC_W_NO_XFP), zp = (flags & LPCC_W_ZERO_POINTS) != 0;
  const bool shared = (flags & LPCC_W_SHARED) != 0;
  const std::vector<Rec> layers = plan(C, D, n_deep, xfp);
  const std::vector<int> own = owners(layers, D - n_deep - 1);
  std::vector<uint8_t> b;
  put32(b, kBlobMagic);
  put32(b, (xfp ? 1u : 2u) | (shared ? 0x100u : 0u));
  put32(b, (uint32_t)C);
  put32(b, (uint32_t)D);
  put32(b, (uint32_t)n_deep);
  put32(b, (uint32_t)layers.size());
  put32(b, (uint32_t)seed);
  put32(b, (uint32_t)(seed >> 32));
  uint64_t ctr = 0;
  for (size_t li = 0; li < layers.size(); li++) {
    const Rec& L = layers[li];
    const int64_t nW = (int64_t)L.taps * L.cin * L.cout;
    // draws ctr+1 .. ctr+nW+cout+2: weights, biases, two zero points
    const uint64_t first = ctr;
    ctr += (uint64_t)(nW + L.cout + 2);
    auto hi = [&](int64_t i) { return (int64_t)(splitmix(seed, first + 1 + (uint64_t)i) >> 33); };
    int64_t m_pos = unit_gain_multiplier((int64_t)L.taps * L.cin);
    if (L.kind == lpcc::K_FC2) m_pos = (3 * m_pos) >> 2;  // logits mostly inside int8
    const bool relu = L.kind == lpcc::K_EMB || L.kind == lpcc::K_DOWN || L.kind == lpcc::K_CONV1 ||
                      L.kind == lpcc::K_FC1;
    const bool prelu = L.kind == lpcc::K_UP;
    const int64_t m_neg = relu ? 0 : (prelu ? (m_pos * 64) >> 8 : m_pos);
    const int32_t z_in = zp ? (int32_t)(hi(nW + L.cout) % 17) - 8 : 0;
    const int32_t z_out = zp ? (int32_t)(hi(nW + L.cout + 1) % 17) - 8 : 0;
    for (int v : {L.kind, L.depth, L.j, L.taps, L.cin, L.cout}) put32(b, (uint32_t)v);
    put32(b, (uint32_t)m_pos);
    put32(b, (uint32_t)m_neg);
    put32(b, 24u);
    put32(b, (uint32_t)z_in);
    put32(b, (uint32_t)z_out);
    if (shared) put32(b, (uint32_t)own[li]);
    for (int o = 0; o < L.cout; o++) put32(b, (uint32_t)(int32_t)(hi(nW + o) % 8193 - 4096));
    if (!shared || own[li] == (int)li)
      for (int64_t i = 0; i < nW; i++) b.push_back((uint8_t)(int8_t)(hi(i) % 255 - 127));
    while (b.size() % 4) b.push_back(0);
  }
  *len = b.size();
  if (!blob || cap < b.size()) return LPCC_E_CAPACITY;
  memcpy(blob, b.data(), b.size());
  return LPCC_OK;
}
