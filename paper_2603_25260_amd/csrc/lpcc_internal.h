// Internal declarations of the gfx950 library: device descriptors shared by
// the kernels and the host runtime.  Integer arithmetic only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/lpcc.h"

namespace lpcc {

constexpr int kMaxD = 21;
constexpr int kNSym = 255;
constexpr int kTaps3 = 27;

enum LayerKind { K_EMB = 1, K_DOWN, K_CONV1, K_CONV2, K_SKIP, K_UP, K_FC1, K_FC2 };

// One layer as the kernels see it.  Weights are packed for the B operand of
// v_mfma_i32_16x16x64_i8: for k-step s (64 input rows k) and column block nb
// (16 outputs) lane l holds 16 bytes W[64 s + 16 (l/16) + i][16 nb + l%16],
// i = 0..15, zero-padded beyond K = taps*cin and cout.
struct LayerDev {
  const int8_t* Wp;     // packed weights, Kpad x Npad bytes
  const int8_t* Wr;     // row-major W[taps][cin][cout] (VALU paths)
  const int32_t* bias;  // [Npad]; dense layers carry -z_in * colsum folded in
  const int32_t* zc;    // [taps][Npad] = -z_in * sum_c W[t][c][o] for sparse layers, or null
  int32_t m_pos, m_neg;  // multipliers (with r = 0 at most 256: the same function)
  int32_t r, z_out;
  int32_t taps, cin, cout;
  int32_t ksteps;       // Kpad / 64
  int32_t npad;
  int32_t a_lo, a_hi;   // accumulator range outside which the output saturates
  int32_t rq24;         // 1: |a| and m below 2^23 and a m + rnd inside int32 on [a_lo, a_hi]
  int64_t rnd;          // 2^(r-1) for r > 0, else 0 (half-up rounding term)
};

// Requantisation of an int32 accumulator (Eq. 14): sign-selected multiplier,
// 64-bit product, round half up, arithmetic shift, zero point, clamp to int8.
// The output is monotone in the accumulator and saturates outside
// [a_lo, a_hi] (derived on the host from m, r and z_out), so the accumulator
// is clamped to that range first; inside it the shifted product is far below
// 2^31, and the zero point and the final clamp are 32-bit operations.
__device__ __forceinline__ int requant_l(int acc, const LayerDev& L) {
  const int a = min(max(acc, L.a_lo), L.a_hi);
  const long long m = a >= 0 ? L.m_pos : L.m_neg;
  const int p = (int)(((long long)a * m + L.rnd) >> L.r);
  return min(max(p + L.z_out, -128), 127);
}

// The same function for layers with rq24 set: a 24-bit signed multiply-add
// gives a m + rnd exactly, so no 64-bit product is needed.
__device__ __forceinline__ int requant_l24(int acc, const LayerDev& L) {
  const int a = min(max(acc, L.a_lo), L.a_hi);
  const int m = a >= 0 ? L.m_pos : L.m_neg;
  const int p = (__mul24(a, m) + (int)L.rnd) >> L.r;
  return min(max(p + L.z_out, -128), 127);
}

// The same for identity layers (m_pos = m_neg, checked on the host): no
// sign-dependent multiplier.
__device__ __forceinline__ int requant_id24(int acc, const LayerDev& L) {
  const int a = min(max(acc, L.a_lo), L.a_hi);
  const int p = (__mul24(a, L.m_pos) + (int)L.rnd) >> L.r;
  return min(max(p + L.z_out, -128), 127);
}

// The same for identity layers whose zero point is folded into the rounding
// term, rndz = rnd + z_out 2^r (a m + rndz inside int32 on [a_lo, a_hi],
// checked on the host): floor((x + z 2^r) / 2^r) = floor(x / 2^r) + z.
__device__ __forceinline__ int requant_idz24(int acc, const LayerDev& L, int rndz) {
  const int a = min(max(acc, L.a_lo), L.a_hi);
  return min(max((__mul24(a, L.m_pos) + rndz) >> L.r, -128), 127);
}

typedef int v4i __attribute__((ext_vector_type(4)));

// Every device array is global memory.  Pointers that arrive inside
// descriptor structs lose that fact, and the compiler would fall back to
// FLAT accesses (which also count against the LDS counter, so every LDS wait
// would drain all outstanding memory loads); gp() restores the address space.
#define GAS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GAS T* gp(const T* p) { return (const GAS T*)p; }
template <class T>
__device__ __forceinline__ GAS T* gp(T* p) { return (GAS T*)p; }

// A layer descriptor read from global memory, field by field
__device__ __forceinline__ LayerDev load_layer(const LayerDev* p) {
  const GAS LayerDev* q = (const GAS LayerDev*)p;
  LayerDev L;
  L.Wp = q->Wp;
  L.Wr = q->Wr;
  L.bias = q->bias;
  L.zc = q->zc;
  L.m_pos = q->m_pos;
  L.m_neg = q->m_neg;
  L.r = q->r;
  L.z_out = q->z_out;
  L.taps = q->taps;
  L.cin = q->cin;
  L.cout = q->cout;
  L.ksteps = q->ksteps;
  L.npad = q->npad;
  L.a_lo = q->a_lo;
  L.a_hi = q->a_hi;
  L.rq24 = q->rq24;
  L.rnd = q->rnd;
  return L;
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP: shifts by 1, 2,
// 4, 8 within each row of 16 lanes (lanes without a source in the row add
// 0), then lane 15 of rows 0 and 2 is added to rows 1 and 3 and lane 31 to
// rows 2 and 3 (row broadcasts; the rows left out add 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_add_src(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, CTRL < 0x140);
}
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  v += dpp_add_src<0x111, 0xF>(v);
  v += dpp_add_src<0x112, 0xF>(v);
  v += dpp_add_src<0x114, 0xF>(v);
  v += dpp_add_src<0x118, 0xF>(v);
  v += dpp_add_src<0x142, 0xA>(v);
  v += dpp_add_src<0x143, 0xC>(v);
  return v;
}

__device__ __forceinline__ v4i mfma16(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Row-range work items.  A launch covers a list of segments; every block
// works on one tile (segment, first row) of the flattened tile list.
// ---------------------------------------------------------------------------
struct Tile {
  int32_t seg;
  int32_t row0;
};

// Gather-GEMM segment: out[row] = epilogue(sum over taps of in[src(row,t)] W[t])
struct GemmSeg {
  const int8_t* in;        // input rows (channels below `split`)
  int64_t in_stride;       // bytes between input rows
  const int8_t* in2;       // channels from `split` on, when split < cin: [in | in2]
  int64_t in2_stride;
  int32_t split;           // first channel read from in2 (cin when unused)
  int32_t pad_;
  const int32_t* kmap;     // conv: [28][kstride]: 27 tap rows of source rows (-1 = empty), presence masks
  int64_t kstride;
  const uint8_t* ccode;    // down: when set, child c reads row ccode[c] of `in` (a table indexed by code)
  const uint8_t* code;     // down/up: occupancy codes of the parents
  const int32_t* cstart;   // down/up: first child row of each parent
  const LayerDev* L;
  int8_t* out;
  int64_t out_stride;
  const int8_t* resid;     // optional residual added after requantisation
  int64_t resid_stride;
  int32_t rows;
  int32_t child_rows;      // rows of the child depth (bounds of cstart-derived indices)
};

// Predictor segment (fc1 -> fc2 -> integer softmax -> frequencies)
struct PredSeg {
  const int8_t* F;         // [rows][C]
  const uint8_t* code;     // encode: true codes (symbol = code - 1)
  const LayerDev* fc1;
  const LayerDev* fc2;
  uint32_t* sf;            // encode: start | freq << 16 per node
  uint16_t* cdf16;         // decode: cdf[0..254] per node (256 slots)
  int32_t* cdf32;          // level_probs: cdf[0..255] per node
  int32_t rows;
  int32_t pad_;
};

// A launch with a single segment passes it, with its layers, by value in the
// kernel arguments (no dependent descriptor loads before the first data
// load); tile t then covers rows [64 t, 64 t + 64).  Otherwise `one` is 0 and
// blocks read their tile and segment from the descriptor arrays.
struct GemmArg {
  GemmSeg seg;
  LayerDev L;
  int32_t one;
  int32_t pad_;
};
struct PredArg {
  PredSeg seg;
  LayerDev fc1, fc2;
  int32_t one;
  int32_t rq24;  // 2: every segment's logit layer is an identity layer with rq24 set whose
                 // zero point folds into the rounding term (requant_idz24); else 0
};

// Coordinate hash and 3x3x3 neighbour table of one depth j; several depths
// share one launch, each starting at its own block.
struct HashJob {
  const uint64_t* keys;    // V_j (frame tag above bit 3j)
  uint64_t* table;         // 16-byte slots {u64 key, i32 row}; empty keys are all ones
  int32_t* kmap;           // [27][kstride]
  int64_t n;
  int64_t kstride;
  uint64_t mask;           // table slots - 1
  int32_t j;
  int32_t blk_insert;      // first block of this depth in the insertion launch
  int32_t blk_kmap;        // first block of this depth in the neighbour launch
  int32_t pad_;
};

// Range-coder chunk: nodes [begin, begin+count) of one (frame, depth)
struct Chunk {
  int64_t node0;           // index into the per-call node arrays
  int32_t count;
  int32_t pad_;
  int64_t scratch;         // byte offset of this chunk's scratch / payload
};

// Device-side error bits
enum : uint32_t { ERR_COORD = 1u, ERR_CORRUPT = 2u, ERR_COUNT = 4u, ERR_ACC = 8u, ERR_SORT = 16u };

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Morton keys and their LSD radix sort (Sec. S3.2: coordinates sorted in
// Morton order).  Keys are sorted on bits [0, end_bit) in passes of at most
// 8 bits, tiles of kSortTile keys; hist is [passes][tiles][256] per-tile digit
// counts (zeroed first), totals [passes][256] digit counts of all keys.
// ---------------------------------------------------------------------------
constexpr int kSortItems = 8;
constexpr int kSortTile = 256 * kSortItems;
constexpr int kSortFusedTiles = 64;  // up to this many tiles a pass scans its own offsets
constexpr int kMortonGroup = 16;     // frames per Morton launch (passed by value)
struct SortPasses {
  int32_t n;
  int32_t shift[8];
  int32_t bits[8];
};
SortPasses sort_passes(int end_bit);
struct MortonFrames {
  const int32_t* xyz[kMortonGroup];  // device coordinates of each frame
  int64_t start[kMortonGroup + 1];   // key range of each frame (start[nf] = end)
  int32_t nf;                        // frames of this launch
  int32_t f0;                        // index of the first (frame tag, error word)
};
// keys of the frames' points (frame tag f << 3D), their per-tile digit
// counts of pass 0 and the digit totals of every pass
hipError_t launch_morton_sort0(const MortonFrames& mf, int D, uint64_t* keys, uint32_t* err, const SortPasses& sp,
                               uint32_t* hist, uint32_t* totals, hipStream_t s);
// pass p: kin -> kout, stable on the pass's digit (for p > 0 the pass first
// counts its digits per tile of kin into hist); ERR_SORT in *err on an
// impossible rank
hipError_t launch_sort_pass(const uint64_t* kin, uint64_t* kout, int64_t n, const SortPasses& sp, int p,
                            uint32_t* hist, const uint32_t* totals, uint32_t* err, hipStream_t s);
// Octree build over sorted keys (frame id in bits >= 3D).
hipError_t launch_level_hist(const uint64_t* keys, int64_t n, int D, int tile, uint32_t* hist,
                             hipStream_t s);
hipError_t launch_level_scan(uint32_t* hist, int nblocks, int D, uint32_t* totals, hipStream_t s);
struct LevelOut {
  uint64_t* key[kMaxD + 1];
  uint8_t* code[kMaxD + 1];
  int32_t* cstart[kMaxD + 1];
  uint32_t* frame_off;  // [frames][D+1]: first node of every frame per depth
};
// (also writes the sentinel cstart[d][N_d] = N_{d+1} of every depth)
hipError_t launch_level_write(const uint64_t* keys, int64_t n, int D, int tile, const uint32_t* hist,
                              const uint32_t* totals, const LevelOut& lo, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_iota_u64(uint64_t* p, int64_t n, hipStream_t s);  // p[i] = i

hipError_t launch_hash_insert(const uint64_t* keys, int64_t n, uint64_t* table, uint64_t mask, hipStream_t s);
// All jobs' insertions, then all jobs' neighbour tables (two launches); the
// block offsets in `jobs` must match the host copy used for the grid sizes.
constexpr int kHashBlock = 256;
hipError_t launch_hash_multi(const HashJob* jobs_dev, int njobs, int insert_blocks, int kmap_blocks,
                             hipStream_t s);
hipError_t launch_kmap(const uint64_t* keys, int64_t n, int j, const uint64_t* table, uint64_t mask,
                       int32_t* kmap, int64_t kstride, hipStream_t s);
// Neighbour table of a depth (n rows, stride n) from the parents' table
// (np rows, stride np), their codes and first-child rows (with the sentinel
// pcstart[np]); no hash table
hipError_t launch_kmap_tree(const int32_t* pkmap, int64_t np, const uint8_t* pcode, const int32_t* pcstart,
                            int32_t* kmap, int64_t n, hipStream_t s);

// GEMM families; `mode` selects the row source
enum GemmMode { G_CONV = 0, G_DENSE = 1, G_DOWN = 2 };
// rb: 16-row blocks per wave (1, 2 or 4); tiles then cover 64 * rb rows
hipError_t launch_gemm(int mode, int cin, int cout, const GemmSeg* segs_dev, const Tile* tiles_dev,
                       int ntiles, const GemmArg& one, int rb, hipStream_t s);
// the same over every tap (absent neighbours and child slots contribute
// zeros): the dense variant the autotuner weighs against the compacted one
hipError_t launch_gemm_dense(int mode, int cin, int cout, const GemmSeg* segs_dev, const Tile* tiles_dev,
                             int ntiles, const GemmArg& one, int rb, hipStream_t s);
hipError_t launch_up(int C, const GemmSeg* segs_dev, const Tile* tiles_dev, int ntiles, const GemmArg& one,
                     int rb, hipStream_t s);
// the same over the occupied children only; tiles of P = 128 or 512 parents
hipError_t launch_up_cx(int C, const GemmSeg* segs_dev, const Tile* tiles_dev, int ntiles, const GemmArg& one,
                        int P, hipStream_t s);
// child convolution (C -> C) over the occupied children only; tiles of P = 64
// or 128 parents
hipError_t launch_down_cx(int C, const GemmSeg* segs_dev, const Tile* tiles_dev, int ntiles, const GemmArg& one,
                          int P, hipStream_t s);
// tile of the compacted child-slot kernels: the large one once a launch has
// this many of its blocks, else the small one (more blocks in flight)
constexpr int kSlotTileBlocks = 512;
hipError_t launch_emb(const GemmSeg* segs_dev, const Tile* tiles_dev, int ntiles, int C, const GemmArg& one,
                      hipStream_t s);
// single-segment predictor launches up to this many rows take 4 rows per wave
constexpr int kPredSmall = 8192;
hipError_t launch_predict(int C, int mode, const PredSeg* segs_dev, const Tile* tiles_dev, int ntiles,
                          const int32_t* lut, const PredArg& one, hipStream_t s);

hipError_t launch_rc_encode(const Chunk* chunks, int nchunks, const uint32_t* sf, uint8_t* scratch,
                            uint32_t* lens, hipStream_t s);
hipError_t launch_rc_pack(const Chunk* chunks, int nchunks, const uint8_t* scratch, const uint32_t* lens,
                          uint8_t* const* dst, hipStream_t s);
// One frame's stream in device memory: output, capacity, its first chunk,
// the offset of its chunk-length table and the header size.
struct PackFrame {
  uint8_t* out;
  uint64_t cap;
  uint32_t first;
  uint32_t pre;
  uint64_t hsz;
};
// Payloads and 16-bit chunk lengths placed straight into the frames' device
// outputs (each chunk after the header and its frame's earlier chunks);
// nothing at or past a frame's capacity is written.
hipError_t launch_rc_pack_dev(const Chunk* chunks, int nchunks, const int32_t* frame_of, const PackFrame* frames,
                              const uint8_t* scratch, const uint32_t* lens, hipStream_t s);
// csum (optional): per chunk, the number of children its decoded codes announce
hipError_t launch_rc_decode_sized(const Chunk* chunks, int nchunks, const uint8_t* payload, const uint16_t* cdf16,
                                  uint8_t* codes, uint32_t* csum, uint32_t* err, size_t max_len, hipStream_t s);
// Child expansion by decoded chunk (one block per chunk) from the chunks'
// child counts: keys of V_{d+1}, first-child rows, and, when table is not
// null, insertion of the children into the hash table of depth d+1.
hipError_t launch_expand_chunks(const Chunk* chunks, int nchunks, const uint64_t* pkeys, const uint8_t* codes,
                                int64_t n, uint32_t* csum, uint64_t* ckeys, int32_t* cstart,
                                int64_t n_child_expected, uint64_t* table, uint64_t mask, uint32_t* err,
                                hipStream_t s);
hipError_t launch_keys_to_xyz(const uint64_t* keys, int64_t n, int D, int32_t* xyz, hipStream_t s);

// ---------------------------------------------------------------------------
// Workspace accounting (host): upper bounds of the three arenas (octree,
// model, descriptors) a call needs, computed by the same carving code the
// calls use, and the serving engine's hooks into a context.
// ---------------------------------------------------------------------------
void encode_workspace_bound(const lpcc_model* m, int nf, const int64_t* n, int cl, bool host_in, size_t out[3]);
// N[f]: the D + 1 node counts of stream f (its header), cl[f] its chunk size
void decode_workspace_bound(const lpcc_model* m, int nf, const int64_t* const* N, const int* cl, size_t out[3]);
void ctx_caps(const lpcc_ctx* c, size_t caps[3]);
void ctx_set_budget(lpcc_ctx* c, size_t budget);
void ctx_trim(lpcc_ctx* c);  // frees the arenas (the context stays usable)

// Base geometry: the depths d < nb are coded from the counts of their own
// codes.  Nodes of those depths are addressed as one range: node i of depth
// d is entry start[d] + i; its frame is key >> 3d (the frame tag).
struct BaseLevels {
  const uint64_t* key[kMaxD];
  const uint8_t* code[kMaxD];
  int64_t start[kMaxD + 1];
  const uint32_t* count;  // device node count per depth, or null: entries of
                          // depth d at or beyond count[d] are skipped
  int32_t nb;             // number of base depths
  int32_t nf;             // frames
};
// hist[(f nb + d) 256 + code] += 1 over every base node (hist cleared first)
hipError_t launch_base_hist(const BaseLevels& bl, uint32_t* hist, hipStream_t s);
// encoder: sf[start[d] + i] = {start | freq << 16} of node i's code under the
// table cdf[(f nb + d) 256 ..] (int32 CDF, cdf[0] = 0, cdf[255] = 65536)
hipError_t launch_base_sf(const BaseLevels& bl, const int32_t* cdf, uint32_t* sf, hipStream_t s);
// decoder: the CDF row (u16 [256]) of every node of base depth d, copied from
// rows16[(f nb + d) 256 ..]
hipError_t launch_base_rows(const uint64_t* keys, int64_t n, int d, int nb, int nf, const uint16_t* rows16,
                            uint16_t* cdf16, hipStream_t s);

// ---------------------------------------------------------------------------
// Static workspace of the allocation-free encode entry point (noalloc.hip)
// ---------------------------------------------------------------------------
constexpr size_t kNoallocBytes = (size_t)256 << 20;  // device bytes per device
constexpr size_t kNoallocHost = (size_t)4 << 20;     // pageable host staging per context
// device address of the block on `device` (current), looked up once per
// device; LPCC_E_DEVICE with the reason in *why when the lookup failed
int scratch_setup(int device, char** base, size_t* cap, std::string* why);
// held for a whole allocation-free call: calls on one device share its block
std::mutex& scratch_mutex(int device);

}  // namespace lpcc
