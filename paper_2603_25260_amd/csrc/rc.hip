// Range coder on gfx950: G. N. N. Martin's byte-oriented range coder (1979)
// with a cache byte and carry propagation; 32-bit range, 16-bit totals.  The
// stream of every (frame, depth) is cut into chunks of 2^c nodes that are
// coded independently: encoding runs one lane per chunk (all depths at once),
// decoding one wave per chunk with a wave-wide symbol search over the CDF.
#include "lpcc_internal.h"

namespace lpcc {

// ---------------------------------------------------------------------------
// Encoder: lane per chunk.  Node i of the chunk carries start | freq << 16.
// Output bytes are gathered into 32-bit words before they are stored.
// ---------------------------------------------------------------------------
struct ByteSink {
  uint32_t* out;
  uint32_t pos;
  uint32_t word;
  __device__ __forceinline__ void put(uint32_t b) {
    word |= (b & 0xFFu) << (8 * (pos & 3u));
    if ((pos & 3u) == 3u) {
      out[pos >> 2] = word;
      word = 0;
    }
    pos++;
  }
};

struct RcEnc {
  uint64_t low;
  uint32_t range;
  uint32_t cache;
  uint32_t pending;
  __device__ __forceinline__ void shift_low(ByteSink& o) {
    if (low < 0xFF000000ull || low >= 0x100000000ull) {
      const uint32_t carry = (uint32_t)(low >> 32);
      o.put(cache + carry);
      for (; pending > 1; pending--) o.put(0xFFu + carry);
      pending = 0;
      cache = (uint32_t)((low >> 24) & 0xFFu);
    }
    pending++;
    low = (low & 0x00FFFFFFull) << 8;
  }
  // freq >= 1 always holds for the model's tables; a zero is clamped so that
  // the renormalisation loop always ends
  __device__ __forceinline__ void encode(uint32_t sf, ByteSink& o) {
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
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  const Chunk ch = chunks[c];
  ByteSink o{(uint32_t*)(scratch + ch.scratch), 0u, 0u};
  RcEnc e{0ull, 0xFFFFFFFFu, 0u, 1u};
  const uint32_t* p = sf + ch.node0;
  const int n = ch.count;
  // symbols in groups of 8, the next group loaded while the current is coded
  uint32_t cur[8], nxt[8];
#pragma unroll
  for (int k = 0; k < 8; k++) cur[k] = k < n ? p[k] : 0u;
  for (int base = 0; base < n; base += 8) {
#pragma unroll
    for (int k = 0; k < 8; k++) nxt[k] = base + 8 + k < n ? p[base + 8 + k] : 0u;
#pragma unroll
    for (int k = 0; k < 8; k++)
      if (base + k < n) e.encode(cur[k], o);
#pragma unroll
    for (int k = 0; k < 8; k++) cur[k] = nxt[k];
  }
  for (int k = 0; k < 5; k++) e.shift_low(o);
  if (o.pos & 3u) o.out[o.pos >> 2] = o.word;
  lens[c] = o.pos;
}

hipError_t launch_rc_encode(const Chunk* chunks, int nchunks, const uint32_t* sf, uint8_t* scratch, uint32_t* lens,
                            hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rc_encode, dim3((nchunks + 63) / 64), dim3(64), 0, s, chunks, nchunks, sf, scratch, lens);
  return hipGetLastError();
}

// Payload assembly: chunk c's bytes go to dst[c].
__global__ void k_rc_pack(const Chunk* __restrict__ chunks, const uint8_t* __restrict__ scratch,
                          const uint32_t* __restrict__ lens, uint8_t* const* __restrict__ dst) {
  const int c = blockIdx.x;
  const uint8_t* src = scratch + chunks[c].scratch;
  uint8_t* d = dst[c];
  const uint32_t n = lens[c];
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = src[i];
}

hipError_t launch_rc_pack(const Chunk* chunks, int nchunks, const uint8_t* scratch, const uint32_t* lens,
                          uint8_t* const* dst, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rc_pack, dim3(nchunks), dim3(256), 0, s, chunks, scratch, lens, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Decoder: one wave per chunk.  The chunk's bytes are staged in LDS; lane l
// holds cdf[4l .. 4l+3] of the current node (cdf[255] = 65536 implied).
// The symbol is the number of entries with r * cdf[s] <= code, minus one,
// counted with four ballots.  CDF rows are prefetched 8 nodes ahead.
// Chunk.pad_ carries the payload length in bytes, Chunk.scratch its offset.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint2 ld_row(const uint16_t* cdf16, int64_t node, int lane) {
  return *(const uint2*)(cdf16 + node * 256 + 4 * lane);
}

__global__ __launch_bounds__(64) void k_rc_decode(const Chunk* __restrict__ chunks,
                                                  const uint8_t* __restrict__ payload,
                                                  const uint16_t* __restrict__ cdf16, uint8_t* __restrict__ codes,
                                                  uint32_t* __restrict__ err) {
  extern __shared__ uint8_t buf[];
  const Chunk ch = chunks[blockIdx.x];
  const int lane = threadIdx.x;
  const uint32_t len = (uint32_t)ch.pad_;
  const uint8_t* src = payload + ch.scratch;
  for (uint32_t i = lane; i < len; i += 64) buf[i] = src[i];
  __syncthreads();

  uint32_t range = 0xFFFFFFFFu, code = 0, pos = 0;
  for (int k = 0; k < 5; k++) {
    code = (code << 8) | (pos < len ? (uint32_t)buf[pos] : 0u);
    pos++;
  }
  const int n = ch.count;
  const int64_t node0 = ch.node0;
  uint2 cur[8], nxt[8];
#pragma unroll
  for (int k = 0; k < 8; k++) cur[k] = k < n ? ld_row(cdf16, node0 + k, lane) : make_uint2(0, 0);
  bool bad = false;
  for (int base = 0; base < n && !bad; base += 8) {
#pragma unroll
    for (int k = 0; k < 8; k++)
      nxt[k] = base + 8 + k < n ? ld_row(cdf16, node0 + base + 8 + k, lane) : make_uint2(0, 0);
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (base + k >= n || bad) break;
      const uint32_t c0 = cur[k].x & 0xFFFFu, c1 = cur[k].x >> 16, c2 = cur[k].y & 0xFFFFu;
      const uint32_t c3 = lane == 63 ? 65536u : (cur[k].y >> 16);
      const uint32_t r = range >> 16;
      if ((uint64_t)code >= ((uint64_t)r << 16)) {
        bad = true;
        break;
      }
      const uint64_t b0 = __ballot(r * c0 <= code), b1 = __ballot(r * c1 <= code);
      const uint64_t b2 = __ballot(r * c2 <= code);
      const uint64_t b3 = __ballot(lane != 63 && r * c3 <= code);
      const int s = __popcll(b0) + __popcll(b1) + __popcll(b2) + __popcll(b3) - 1;
      const int es = s & 3, es1 = (s + 1) & 3;
      const uint32_t vs = es == 0 ? c0 : (es == 1 ? c1 : (es == 2 ? c2 : c3));
      const uint32_t vs1 = es1 == 0 ? c0 : (es1 == 1 ? c1 : (es1 == 2 ? c2 : c3));
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)vs, s >> 2);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)vs1, (s + 1) >> 2);
      if (hi <= lo) {  // not a valid CDF row: stop instead of looping
        bad = true;
        break;
      }
      code -= r * lo;
      range = r * (hi - lo);
      while (range < (1u << 24)) {
        code = (code << 8) | (pos < len ? (uint32_t)buf[pos] : 0u);
        pos++;
        range <<= 8;
      }
      if (lane == 0) codes[node0 + base + k] = (uint8_t)(s + 1);
    }
#pragma unroll
    for (int k = 0; k < 8; k++) cur[k] = nxt[k];
  }
  if (bad && lane == 0) atomicOr(err, ERR_CORRUPT);
}

hipError_t launch_rc_decode_sized(const Chunk* chunks, int nchunks, const uint8_t* payload, const uint16_t* cdf16,
                                  uint8_t* codes, uint32_t* err, size_t max_len, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  size_t lds = (max_len + 15) & ~(size_t)15;
  if (lds == 0) lds = 16;
  hipLaunchKernelGGL(k_rc_decode, dim3(nchunks), dim3(64), lds, s, chunks, payload, cdf16, codes, err);
  return hipGetLastError();
}

}  // namespace lpcc
