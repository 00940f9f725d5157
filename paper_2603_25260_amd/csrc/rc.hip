// Range coder on gfx950: G. N. N. Martin's byte-oriented range coder (1979)
// with a cache byte and carry propagation; 32-bit range, 16-bit totals.  The
// stream of every (frame, depth) is cut into chunks of 2^c nodes that are
// coded independently: encoding runs one wave per chunk, or one lane per
// chunk when there are many (all depths at once), decoding one wave per chunk
// with a wave-wide symbol search over the CDF.
#include "lpcc_internal.h"

namespace lpcc {

constexpr int kRcEncodeLanes = 2048;

// ---------------------------------------------------------------------------
// Encoder: one wave per chunk.  The coder state is wave-uniform (scalar
// registers); the node values start | freq << 16 are loaded 64 at a time
// (one per lane, the next 64 in flight) and taken one by one with readlane.
// Each output byte is one vector byte store that every lane issues with the
// same address and value (a single memory transaction), so emitting a byte
// needs no branch and no packing.
// ---------------------------------------------------------------------------
struct WaveSink {
  GAS uint8_t* out;
  uint32_t pos;  // bytes emitted
  __device__ __forceinline__ void put(uint32_t b) {
    out[pos] = (uint8_t)b;
    pos++;
  }
};

struct RcEnc {
  uint64_t low;
  uint32_t range;
  uint32_t cache;
  uint32_t pending;
  template <class Sink>
  __device__ __forceinline__ void shift_low(Sink& o) {
    // low < 2^33: bits 24..32 hold the carry and the top byte; a byte leaves
    // unless they read 0x0FF (one 32-bit scalar compare)
    const uint32_t top = (uint32_t)(low >> 24);
    if (top != 0xFFu) {
      const uint32_t carry = top >> 8;
      o.put(cache + carry);
      for (; pending > 1; pending--) o.put(0xFFu + carry);
      pending = 0;
      cache = top & 0xFFu;
    }
    pending++;
    low = (low & 0x00FFFFFFull) << 8;
  }
  // freq >= 1 always holds for the model's tables; a zero is clamped so that
  // the renormalisation loop always ends
  template <class Sink>
  __device__ __forceinline__ void encode(uint32_t sf, Sink& o) {
    const uint32_t start = sf & 0xFFFFu, freq = (sf >> 16) ? (sf >> 16) : 1u;
    const uint32_t r = range >> 16;
    low += (uint64_t)r * start;
    range = r * freq;
    while (range < (1u << 24)) {
      range <<= 8;
      shift_low(o);
    }
  }
};

__global__ __launch_bounds__(64) void k_rc_encode(const Chunk* __restrict__ chunks, int nch,
                                                  const uint32_t* __restrict__ sf, uint8_t* __restrict__ scratch,
                                                  uint32_t* __restrict__ lens) {
  const int lane = threadIdx.x;
  const Chunk ch = chunks[blockIdx.x];
  WaveSink o{(GAS uint8_t*)(scratch + ch.scratch), 0u};
  RcEnc e{0ull, 0xFFFFFFFFu, 0u, 1u};
  const GAS uint32_t* p = gp(sf) + ch.node0;
  const int n = ch.count;
  uint32_t v = lane < n ? p[lane] : 0u;
  for (int base = 0; base < n; base += 64) {
    // wave-uniform trip count kept in a scalar register
    const int cnt = __builtin_amdgcn_readfirstlane(min(64, n - base));
    const uint32_t vn = base + 64 + lane < n ? p[base + 64 + lane] : 0u;  // next 64 in flight
    for (int k = 0; k < cnt; k++) e.encode((uint32_t)__builtin_amdgcn_readlane((int)v, k), o);
    v = vn;
  }
  for (int k = 0; k < 5; k++) e.shift_low(o);
  if (lane == 0) lens[blockIdx.x] = o.pos;
}

// Encoder for many chunks: one lane per chunk, the coder state in vector
// registers.  The wave-per-chunk form above keeps its state in scalar
// registers, and a compute unit has one scalar unit for all its waves, so
// with thousands of chunks in flight the scalar unit, not the chunks' serial
// chains, sets the time; here 64 chunks advance side by side on the vector
// unit.  Each lane stores its own chunk's bytes.  Same bytes as above.
struct LaneSink {
  GAS uint8_t* out;
  uint32_t pos;
  __device__ __forceinline__ void put(uint32_t b) {
    out[pos] = (uint8_t)b;
    pos++;
  }
};

__global__ __launch_bounds__(64) void k_rc_encode_lanes(const Chunk* __restrict__ chunks, int nch,
                                                        const uint32_t* __restrict__ sf,
                                                        uint8_t* __restrict__ scratch, uint32_t* __restrict__ lens) {
  const int c = (int)blockIdx.x * 64 + (int)threadIdx.x;
  if (c >= nch) return;
  const Chunk ch = chunks[c];
  LaneSink o{(GAS uint8_t*)(scratch + ch.scratch), 0u};
  RcEnc e{0ull, 0xFFFFFFFFu, 0u, 1u};
  const GAS uint32_t* p = gp(sf) + ch.node0;
  const int n = ch.count;
  // symbols in batches of 16, the next batch in flight while one is coded
  constexpr int kB = 16;
  uint32_t cur[kB], nxt[kB];
#pragma unroll
  for (int j = 0; j < kB; j++) cur[j] = j < n ? p[j] : 0u;
  for (int base = 0; base < n; base += kB) {
#pragma unroll
    for (int j = 0; j < kB; j++) nxt[j] = base + kB + j < n ? p[base + kB + j] : 0u;
#pragma unroll
    for (int j = 0; j < kB; j++)
      if (base + j < n) e.encode(cur[j], o);
#pragma unroll
    for (int j = 0; j < kB; j++) cur[j] = nxt[j];
  }
  for (int k = 0; k < 5; k++) e.shift_low(o);
  lens[c] = o.pos;
}

hipError_t launch_rc_encode(const Chunk* chunks, int nchunks, const uint32_t* sf, uint8_t* scratch, uint32_t* lens,
                            hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  // lane per chunk once there are enough chunks to fill many waves
  if (nchunks >= kRcEncodeLanes)
    hipLaunchKernelGGL(k_rc_encode_lanes, dim3((nchunks + 63) / 64), dim3(64), 0, s, chunks, nchunks, sf, scratch,
                       lens);
  else
    hipLaunchKernelGGL(k_rc_encode, dim3(nchunks), dim3(64), 0, s, chunks, nchunks, sf, scratch, lens);
  return hipGetLastError();
}

// Payload assembly: chunk c's bytes go to dst[c].
__global__ void k_rc_pack(const Chunk* __restrict__ chunks, const uint8_t* __restrict__ scratch,
                          const uint32_t* __restrict__ lens, uint8_t* const* __restrict__ dst) {
  const int c = blockIdx.x;
  const uint8_t* src = scratch + chunks[c].scratch;
  uint8_t* d = dst[c];
  const uint32_t n = lens[c];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) gp(d)[i] = src[i];
}

hipError_t launch_rc_pack(const Chunk* chunks, int nchunks, const uint8_t* scratch, const uint32_t* lens,
                          uint8_t* const* dst, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rc_pack, dim3(nchunks), dim3(256), 0, s, chunks, scratch, lens, dst);
  return hipGetLastError();
}

// Placement without a host round trip: block c sums the lengths of its
// frame's earlier chunks itself (a frame has at most a few thousand), writes
// its length into the header's table and copies its bytes; every write is
// checked against the frame's capacity.
__global__ __launch_bounds__(256) void k_rc_pack_dev(const Chunk* __restrict__ chunks,
                                                     const int32_t* __restrict__ frame_of,
                                                     const PackFrame* __restrict__ frames,
                                                     const uint8_t* __restrict__ scratch,
                                                     const uint32_t* __restrict__ lens) {
  __shared__ uint32_t wsum[4];
  const uint32_t c = blockIdx.x;
  const PackFrame F = frames[frame_of[c]];
  const uint32_t n = lens[c];
  uint32_t part = 0;
  for (uint32_t k = F.first + threadIdx.x; k < c; k += 256) part += lens[k];
  part = wave_scan_incl(part);  // lane 63: the wave's sum
  if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = part;
  __syncthreads();
  const uint64_t off = F.hsz + wsum[0] + wsum[1] + wsum[2] + wsum[3];
  GAS uint8_t* out = gp(F.out);
  if (threadIdx.x < 2) {
    const uint64_t p = (uint64_t)F.pre + 2ull * (c - F.first) + threadIdx.x;
    if (p < F.cap) out[p] = (uint8_t)(n >> (8 * threadIdx.x));
  }
  const uint8_t* src = scratch + chunks[c].scratch;
  for (uint32_t i = threadIdx.x; i < n; i += 256)
    if (off + i < F.cap) out[off + i] = src[i];
}

hipError_t launch_rc_pack_dev(const Chunk* chunks, int nchunks, const int32_t* frame_of, const PackFrame* frames,
                              const uint8_t* scratch, const uint32_t* lens, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rc_pack_dev, dim3(nchunks), dim3(256), 0, s, chunks, frame_of, frames, scratch, lens);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Decoder: one wave per chunk.  The chunk's bytes are staged in LDS (zero
// padded: bytes past the end read as 0) and consumed through a dword window.
// CDF rows are loaded kDecBlock at a time straight into registers (one
// memory round trip per block, the next block in flight while this one is
// decoded).  Lane l holds the boundaries b_j = cdf[4l + j], j = 0..3, of the
// current node as two packed words (b_0 b_1 | b_2 b_3), and b_4 is lane l+1's
// b_0.  cdf[255] = 2^16 is stored as 0.  The symbol s is the last index with
// r * cdf[s] <= code (r < 2^16, cdf <= 2^16, so 24-bit multiplies are exact).
// Every lane compares its four entries and selects the packed pair
// (b_j, b_j+1) of the last entry passed; the owning lane is
// popcount(ballot(r * b_0 <= code)) - 1 (lane 0 always qualifies, cdf[0] =
// 0), and one readlane brings the pair to the scalar coder state, where an
// upper boundary of 0 stands for 2^16 (the frequency is taken mod 2^16).  A
// corrupt stream is one where no symbol fits (code >= r * 2^16): lane 63,
// whose b_3 compares as 2^16, then passes all four entries and yields the
// pair (0, 0), so the range becomes 0 and stays 0, which is checked once per
// block.  Decoded codes are collected one per lane and stored kDecBlock at a
// time.  Chunk.pad_ carries the payload length in bytes, Chunk.scratch its
// offset.
// ---------------------------------------------------------------------------
constexpr int kDecBlock = 32;

__device__ __forceinline__ uint2 ld_row(const uint16_t* cdf16, int64_t node, int lane) {
  return *(const uint2*)(cdf16 + node * 256 + 4 * lane);
}

// PW > 0: the payload (at most 64*PW dwords) sits in VGPRs, dword w in lane
// w%64 of register w/64, read with v_readlane; PW = 0 reads it from LDS (long
// chunks).  The renormalisation takes 0, 1 or 2 bytes from a 64-bit buffer
// without branches.
template <int PW>
__global__ __launch_bounds__(64) void k_rc_decode(const Chunk* __restrict__ chunks,
                                                  const uint8_t* __restrict__ payload,
                                                  const uint16_t* __restrict__ cdf16, uint8_t* __restrict__ codes,
                                                  uint32_t* __restrict__ csum, uint32_t* __restrict__ err,
                                                  int lds_words) {
  extern __shared__ uint32_t buf[];
  const Chunk ch = chunks[blockIdx.x];
  const int lane = threadIdx.x;
  const uint32_t len = (uint32_t)ch.pad_;
  const uint8_t* src = payload + ch.scratch;
  const int n = ch.count;
  const int64_t node0 = ch.node0;
  const int last = max(n - 1, 0);
  // rows of the first two blocks in flight before the payload is staged
  uint2 ta[kDecBlock], tb[kDecBlock];
#pragma unroll
  for (int k = 0; k < kDecBlock; k++) ta[k] = ld_row(cdf16, node0 + min(k, last), lane);
#pragma unroll
  for (int k = 0; k < kDecBlock; k++) tb[k] = ld_row(cdf16, node0 + min(kDecBlock + k, last), lane);
  for (int w = lane; w < lds_words; w += 64) {
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t b = 4u * (uint32_t)w + (uint32_t)k;
      if (b < len) v |= (uint32_t)src[b] << (24 - 8 * k);
    }
    buf[w] = v;
  }
  __syncthreads();
  uint32_t pw[PW > 0 ? PW : 1];
#pragma unroll
  for (int j = 0; j < (PW > 0 ? PW : 1); j++) pw[j] = (PW > 0 && 64 * j + lane < lds_words) ? buf[64 * j + lane] : 0u;

  // payload dwords in stream order, big-endian: byte 0 of the stream is the
  // high byte of dword 0
  uint32_t cj = 0, creg = pw[0];
  auto dword = [&](uint32_t w) -> uint32_t {
    if (PW == 0) return (int)w < lds_words ? buf[w] : 0u;
    if ((int)w >= 64 * PW) return 0u;
    if ((w >> 6) != cj) {  // rare: next register of the payload
      cj = w >> 6;
#pragma unroll
      for (int j = 0; j < (PW > 0 ? PW : 1); j++)
        if ((uint32_t)j == cj) creg = pw[j];
    }
    return (uint32_t)__builtin_amdgcn_readlane((int)creg, (int)(w & 63u));
  };
  // bit buffer: the next `nbit` stream bits (whole bytes), first byte in bits 63..56
  uint64_t bb = 0;
  uint32_t nbit = 0, wnext = 0;
  auto refill = [&]() {  // append one dword (4 bytes, stream order); nbit < 32
    bb |= (uint64_t)dword(wnext++) << (32 - nbit);
    nbit += 32;
  };
  refill();
  refill();
  // the first 5 bytes: the first is always 0 and shifts out of 32 bits
  uint32_t code = (uint32_t)(bb >> 24);
  bb <<= 40;
  nbit -= 40;
  uint32_t range = 0xFFFFFFFFu;

  uint32_t kids = 0;  // children announced by the codes this lane stored
  // high half of b_3 for the compare: lane 63's b_3 = cdf[255] is stored as 0
  // and compares as 2^16
  const uint32_t b3hi = lane == 63 ? 1u : 0u;
  bool bad = false;

  // one symbol from the row (b_0 b_1 | b_2 b_3) of this lane; its code goes to lane k of cv
  auto symbol = [&](const uint2 row, const int k, uint32_t& cv) {
    const uint32_t x = row.x, y = row.y;
    // lane+1's (b_0, b_1); 0 in lane 63 (bound_ctrl: out-of-range source reads 0)
    const uint32_t nx = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x130, 0xF, 0xF, true);
    const uint32_t r = range >> 16;
    const uint32_t b3 = __builtin_amdgcn_alignbit(b3hi, y, 16);
    const bool m0 = __umul24(r, x & 0xFFFFu) <= code;
    const bool m1 = __umul24(r, x >> 16) <= code;
    const bool m2 = __umul24(r, y & 0xFFFFu) <= code;
    const bool m3 = __umul24(r, b3) <= code;
    // (b_j, b_{j+1}) packed low/high for the last entry j passed
    // (bytes 2, 3 of the low word, bytes 0, 1 of the high word)
    const uint32_t q1 = __builtin_amdgcn_perm(y, x, 0x05040302u);
    const uint32_t q3 = __builtin_amdgcn_perm(nx, y, 0x05040302u);
    uint32_t q = m1 ? q1 : x;
    q = m2 ? y : q;
    q = m3 ? q3 : q;
    const int L = (int)__popcll(__ballot(m0)) - 1;
    const uint32_t Q = (uint32_t)__builtin_amdgcn_readlane((int)q, L);
    const uint32_t lo = Q & 0xFFFFu;
    // an upper boundary stored as 0 is 2^16; both 0 on a corrupt stream
    const uint32_t freq = ((Q >> 16) - lo) & 0xFFFFu;
    code -= r * lo;
    range = r * freq;
    // renormalise: a valid step leaves range >= 2^8, so take 0, 1 or 2 bytes
    const uint32_t sh = (uint32_t)__builtin_clz(range | 1u) & 24u;
    // (code, top 4 buffered bytes) as one 64-bit register pair, shifted up
    const uint64_t cx = __builtin_bit_cast(uint64_t, make_uint2((uint32_t)(bb >> 32), code));
    code = (uint32_t)((cx << sh) >> 32);
    bb <<= sh;
    nbit -= sh;
    range <<= sh;
    // the symbol is resolved later from (lo, owning lane): lane k keeps them
    const uint32_t pk = lo | ((uint32_t)L << 16);
    cv = lane == k ? pk : cv;
  };
  // one block of up to kDecBlock symbols from the rows in t (fully unrolled:
  // row k is register t[k]); then t is reloaded with the block two ahead.
  // A symbol takes at most 2 bytes: 4 buffered bytes cover a pair.
  // Symbols of a block are resolved one block later: lane k holds (lo, L) of
  // symbol k, reads its node's entries b_0..b_3 of lane L (the read is issued
  // at the end of the block and used at the end of the next one) and finds
  // j with b_j = lo (the entries of a row are distinct; cdf[255] is stored as
  // 0 but is never a lower boundary of a valid symbol): code = 4 L + j + 1.
  uint32_t pend_pk = 0;
  uint2 pend_e = make_uint2(0u, 0u);
  int pend_base = 0, pend_cnt = 0;  // pend_cnt = 0: nothing pending
  auto resolve = [&]() {
    if (pend_cnt > 0 && lane < pend_cnt) {
      const uint32_t lo = pend_pk & 0xFFFFu, L = pend_pk >> 16;
      const uint32_t j = lo == (pend_e.x >> 16) ? 1u : (lo == (pend_e.y & 0xFFFFu) ? 2u : (lo == (pend_e.y >> 16) ? 3u : 0u));
      const uint32_t cv = 4u * L + j + 1u;
      codes[node0 + pend_base + lane] = (uint8_t)cv;
      kids += __popc(cv & 0xFFu);
    }
    pend_cnt = 0;
  };
  auto block = [&](uint2 (&t)[kDecBlock], int base) {
    const int cnt = min(kDecBlock, n - base);
    uint32_t cv = 0;  // (lo, owning lane) of symbol k of this block in lane k
#pragma unroll
    for (int k = 0; k < kDecBlock; k++) {
      if (k < cnt) {
        if ((k & 1) == 0 && nbit < 32u) refill();
        symbol(t[k], k, cv);
      }
    }
    bad = range == 0u;
    resolve();  // the previous block (decoded before any corruption here)
    if (!bad) {
      pend_pk = cv;
      pend_base = base;
      pend_cnt = cnt;
      const int64_t node = node0 + base + min(lane, cnt - 1);
      pend_e = *(const uint2*)(cdf16 + node * 256 + 4 * (cv >> 16 & 63u));
    }
    const int nbk = base + 2 * kDecBlock;
#pragma unroll
    for (int k = 0; k < kDecBlock; k++) t[k] = ld_row(cdf16, node0 + min(nbk + k, last), lane);
  };
  for (int base = 0; base < n && !bad; base += 2 * kDecBlock) {
    block(ta, base);
    if (base + kDecBlock < n && !bad) block(tb, base + kDecBlock);
  }
  resolve();
  if (bad && lane == 0) atomicOr(err, ERR_CORRUPT);
  if (csum != nullptr) {
    kids = wave_scan_incl(kids);  // lane 63: the chunk's child count
    if (lane == 63) csum[blockIdx.x] = kids;
  }
}

hipError_t launch_rc_decode_sized(const Chunk* chunks, int nchunks, const uint8_t* payload, const uint16_t* cdf16,
                                  uint8_t* codes, uint32_t* csum, uint32_t* err, size_t max_len, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  const int words = (int)((max_len + 3) / 4) + 4;
  if (words <= 64 * 12) {
    hipLaunchKernelGGL((k_rc_decode<12>), dim3(nchunks), dim3(64), (size_t)words * 4, s, chunks, payload, cdf16,
                       codes, csum, err, words);
  } else {
    hipLaunchKernelGGL((k_rc_decode<0>), dim3(nchunks), dim3(64), (size_t)words * 4, s, chunks, payload, cdf16,
                       codes, csum, err, words);
  }
  return hipGetLastError();
}

}  // namespace lpcc
