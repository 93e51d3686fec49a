// pq_scan_kernels.hip -- kernels of one scan (everything pq_scan enqueues).
//
//   k_snappy       Snappy page bodies -> workspace (one wave per page)
//   k_prep         validity edge words cleared / REQUIRED validity set to ones
//   k_dict         dictionary pages -> device dictionaries
//   k_prepass      per-tile DELTA sums and string byte counts
//   k_tile_scan    exclusive prefix over tiles (DELTA carries, string bases)
//   k_decode_fixed definition levels, PLAIN / dictionary / DELTA values
//   k_decode_str   definition levels, PLAIN / dictionary strings
//
// Work unit of the decode kernels: one TILE_ROWS-row tile of one page per
// 256-thread workgroup, entered through the tile index built at open.  Each
// tile first copies the byte ranges of its level and value streams into LDS
// with one coalesced 16-byte-per-lane load; a single wave then walks the
// run / block headers over the staged bytes, 64 candidate header positions
// at a time (each lane parses the header that would start at its byte; the
// real chain is followed with readlane), and all threads expand the runs.
#include <hip/hip_runtime.h>

#include "pq_device.hpp"
#include "pq_internal.h"

namespace pqk {

constexpr int WG = 256;
constexpr int NWAVES = WG / 64;
constexpr int TR = TILE_ROWS;        // rows per tile
constexpr int NWORDS = TR / 32;      // validity words per tile
constexpr int RUNCAP = 512;          // run-table entries per batch
constexpr int STAGE_DEF = 2048;      // bytes of staged level stream
constexpr int STAGE_VAL = 9216;      // bytes of staged value stream
constexpr int DBLK_CAP = 24;         // DELTA blocks per tile (TR / 128 + 2)
constexpr int DMINI_MAX = 16;

struct Run {
  int32_t vstart;  // first value (tile-relative; negative for a run entered mid-way)
  uint32_t nbp;    // values | (bit-packed << 31)
  uint64_t pay;    // bit-packed: bit position of the payload in the source; RLE: the value
};

struct DBlock {
  int32_t dfirst;   // first delta of the block, relative to the tile's first delta
  uint32_t nmb;
  int64_t min_delta;
  uint64_t bit0;    // bit position (in the source) of miniblock 0's body
  uint32_t woff[DMINI_MAX];
  uint8_t w[DMINI_MAX];
};

struct Streams {
  const uint8_t* dbase;
  uint64_t doff, dend;
  const uint8_t* vbase;
  uint64_t voff, vend;
};

__device__ __forceinline__ Streams page_streams(const PageDev& pg, const ColScan& cs, const uint8_t* file, uint8_t* ws) {
  Streams s;
  const uint8_t* sb = ws + cs.ws_scratch;
  if (pg.flags & 1) { s.dbase = sb; s.doff = pg.def_off - cs.scratch_base; }
  else { s.dbase = file; s.doff = pg.def_off; }
  s.dend = s.doff + (uint64_t)pg.def_len;
  if (pg.flags & 2) { s.vbase = sb; s.voff = pg.val_off - cs.scratch_base; }
  else { s.vbase = file; s.voff = pg.val_off; }
  s.vend = s.voff + pg.val_len;
  return s;
}

__device__ __forceinline__ void find_segment(const SegTable& seg, uint32_t wg, uint32_t& csi, uint32_t& t) {
  int k = 0;
  for (int j = 1; j < seg.n; ++j)
    if (seg.s[j].wg0 <= wg) k = j;
  csi = seg.s[k].cs;
  t = seg.s[k].t0 + (wg - seg.s[k].wg0);
}

// ---------------------------------------------------------------------------
// byte sources: staged LDS copy, or global memory (fallback)
// ---------------------------------------------------------------------------
struct LSrc {
  const uint8_t* p;  // 16-byte aligned LDS buffer
  uint32_t len;      // staged bytes (multiple of 16)
  __device__ __forceinline__ uint32_t byte(uint64_t i) const { return i < len ? (uint32_t)p[i] : 0u; }
  __device__ __forceinline__ uint64_t bits(uint64_t bit, uint32_t w) const {
    if (w == 0) return 0;
    const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
    const uint64_t dw = bit >> 5;
    const uint32_t sh = (uint32_t)(bit & 31);
    const uint64_t nd = len >> 2;
    const uint64_t lo = dw < nd ? q[dw] : 0u;
    const uint64_t mid = dw + 1 < nd ? q[dw + 1] : 0u;
    uint64_t v = (lo | (mid << 32)) >> sh;
    if (sh + w > 64) v |= (uint64_t)(dw + 2 < nd ? q[dw + 2] : 0u) << (64 - sh);
    return w == 64 ? v : (v & ((1ull << w) - 1));
  }
};
struct GSrc {
  const uint8_t* base;  // 16-byte aligned
  uint64_t origin;      // absolute offset of position 0
  uint64_t len;
  __device__ __forceinline__ uint32_t byte(uint64_t i) const { return i < len ? (uint32_t)base[origin + i] : 0u; }
  __device__ __forceinline__ uint64_t bits(uint64_t bit, uint32_t w) const { return get_bits(base, origin * 8 + bit, w); }
};

// Copies bytes [abs_begin, abs_end) of `base` into LDS, starting at the
// 16-byte boundary at or below abs_begin.  Uniform result: false if they do
// not fit `cap` (nothing copied).
__device__ __forceinline__ bool stage(uint8_t* lds, uint32_t cap, const uint8_t* base, uint64_t abs_begin,
                                      uint64_t abs_end, uint64_t& origin, uint32_t& len) {
  origin = abs_begin & ~15ull;
  const uint64_t n16 = (abs_end - origin + 15) >> 4;
  if (abs_end <= abs_begin) { len = 0; return true; }
  if (n16 * 16 > cap) return false;
  const uint4* src = reinterpret_cast<const uint4*>(base + origin);
  uint4* dst = reinterpret_cast<uint4*>(lds);
  for (uint32_t i = threadIdx.x; i < (uint32_t)n16; i += WG) dst[i] = src[i];
  len = (uint32_t)(n16 * 16);
  return true;
}

// ---------------------------------------------------------------------------
// workgroup scans
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// exclusive scan of one u64 per thread over the workgroup (wrapping); the
// total goes to *total.  Contains two barriers.
__device__ __forceinline__ uint64_t wg_excl_scan_u64(uint64_t v, uint64_t* s_tmp, uint64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = wave_incl_scan_u64(v);
  if (lane == 63) s_tmp[wave] = inc;
  __syncthreads();
  uint64_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NWAVES; ++k) {
    uint64_t x = s_tmp[k];
    if (k < wave) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// ---------------------------------------------------------------------------
// RLE / bit-packed hybrid: run-header walk by one wave
// ---------------------------------------------------------------------------
// Follows the chain of run headers from position `cur` (whose run starts at
// value `v`, tile-relative) until value `count` is covered or `cap` runs are
// recorded.  Each lane parses the header that would start at cur + lane; the
// wave then follows the real chain through those 64 candidates with
// readlane, and the header lanes write their runs (with prefix-summed value
// starts) and the first-run marks of the 32-value words their runs cover.
// Uniform in/out: cur, v.  Returns the runs recorded; *bad on a malformed
// header (or levels > 1).
template <class Src>
__device__ uint32_t wave_walk(const Src& src, uint64_t& cur, int64_t& v, uint32_t count, uint32_t w, bool levels,
                              Run* runs, uint32_t cap, uint32_t* s_first, bool& bad) {
  const int lane = threadIdx.x & 63;
  uint32_t nr = 0;
  while (v < (int64_t)count && nr < cap) {
    const uint64_t p = cur + (uint64_t)lane;
    // candidate header at p
    uint64_t h = 0;
    uint32_t hl = 0;
    bool ok = false;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint32_t b = src.byte(p + k);
      h |= (uint64_t)(b & 0x7f) << (7 * k);
      if (!(b & 0x80)) { hl = k + 1; ok = true; break; }
    }
    const bool isbp = h & 1;
    const uint64_t g = h >> 1;
    uint64_t cnt, plen;
    uint32_t val = 0;
    if (isbp) {
      cnt = g * 8;
      plen = g * w;
    } else {
      cnt = g;
      plen = (w + 7) / 8;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((uint32_t)k < plen) val |= src.byte(p + hl + k) << (8 * k);
      if (levels && val > 1) ok = false;
    }
    if (cnt > 0x7fffffffull || plen > 0x7fffffffull || p + hl > src.len) ok = false;
    const uint32_t adv = (uint32_t)(hl + plen);
    const uint32_t c32 = (uint32_t)cnt;
    const uint32_t pay_end = (uint32_t)min(p + hl, (uint64_t)0xffffffffull);  // payload start
    // follow the chain
    uint32_t l = 0;
    uint64_t mask = 0;
    const int64_t v0 = v;
    uint32_t nwin = 0;
    while (l < 64 && v < (int64_t)count && nr + nwin < cap) {
      if (!__builtin_amdgcn_readlane((int)ok, (int)l)) { bad = true; break; }
      const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)c32, (int)l);
      {
        // the part of this run the tile needs must lie inside the source
        const uint64_t need = min((uint64_t)c, (uint64_t)((int64_t)count - v));
        const uint64_t ps = (uint32_t)__builtin_amdgcn_readlane((int)pay_end, (int)l);
        const bool rbp = (uint32_t)__builtin_amdgcn_readlane((int)isbp, (int)l) != 0;
        const uint64_t nb = rbp ? (need * w + 7) / 8 : (uint64_t)(w + 7) / 8;
        if (ps + nb > src.len) { bad = true; break; }
      }
      if (c) { mask |= 1ull << l; ++nwin; }
      v += c;
      l += (uint32_t)__builtin_amdgcn_readlane((int)adv, (int)l);
    }
    if (bad) return nr;
    // record the runs of this window
    const bool me = (mask >> lane) & 1ull;
    const uint64_t cm = me ? (uint64_t)c32 : 0ull;
    const uint64_t incl = wave_incl_scan_u64(cm);
    if (me) {
      const uint32_t k = nr + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
      const int64_t vs = v0 + (int64_t)(incl - cm);
      Run R;
      R.vstart = (int32_t)vs;
      R.nbp = c32 | (isbp ? 0x80000000u : 0u);
      R.pay = isbp ? (p + hl) * 8 : (uint64_t)val;
      runs[k] = R;
      int64_t j = vs <= 0 ? 0 : (vs + 31) >> 5;
      for (; j < NWORDS && j * 32 < vs + (int64_t)c32; ++j) s_first[j] = k;
    }
    nr += nwin;
    cur += l;
  }
  return nr;
}

// Expands the definition levels of one batch [lo, hi) of tile rows into the
// LDS validity words (one thread per 32-row word).
template <class Src>
__device__ void expand_levels(const Src& src, const Run* runs, const uint32_t* s_first, uint32_t lo, uint32_t hi,
                              uint32_t* s_valid) {
  const uint32_t w0 = lo >> 5, w1 = (hi + 31) >> 5;
  for (uint32_t j = w0 + threadIdx.x; j < w1; j += WG) {
    uint32_t r = max(j * 32, lo);
    const uint32_t re = min(j * 32 + 32, hi);
    uint32_t k = (j * 32 < lo) ? 0u : s_first[j];
    uint32_t word = 0;
    while (r < re) {
      const Run R = runs[k];
      const uint32_t n = R.nbp & 0x7fffffffu;
      const uint32_t e = min(re, (uint32_t)((int64_t)R.vstart + n));
      const uint32_t c = e - r;
      uint32_t b;
      if (R.nbp >> 31) b = (uint32_t)src.bits(R.pay + (uint64_t)((int64_t)r - R.vstart), c);
      else b = R.pay ? (c == 32 ? 0xffffffffu : ((1u << c) - 1)) : 0u;
      word |= b << (r - j * 32);
      r = e;
      ++k;
    }
    s_valid[j] |= word;
  }
}

// Decodes values [lo, hi) of a batch of an index stream (bit width w) into
// idx[]; flags indices >= dn.
template <class Src>
__device__ void expand_indices(const Src& src, const Run* runs, uint32_t nr, const uint32_t* s_first, uint32_t lo,
                               uint32_t hi, uint32_t w, uint32_t dn, uint32_t* idx, uint32_t* s_flag) {
  for (uint32_t i = lo + threadIdx.x; i < hi; i += WG) {
    const uint32_t j = i >> 5;
    uint32_t k = (j * 32 < lo) ? 0u : s_first[j];
    while (k + 1 < nr && runs[k + 1].vstart <= (int32_t)i) ++k;
    const Run R = runs[k];
    uint32_t x = (R.nbp >> 31) ? (uint32_t)src.bits(R.pay + (uint64_t)((int64_t)i - R.vstart) * w, w) : (uint32_t)R.pay;
    if (x >= dn) { *s_flag = 1; x = 0; }
    idx[i] = x;
  }
}

// Walks + expands a whole hybrid stream segment of `count` values (batches
// of RUNCAP runs).  MODE 0: definition levels into s_valid; MODE 1:
// dictionary indices into idx.  Returns false on a malformed stream.
template <int MODE, class Src>
__device__ bool decode_hybrid(const Src& src, uint64_t pos, uint32_t skip, uint32_t count, uint32_t w, Run* runs,
                              uint32_t* s_first, uint32_t* s_valid, uint32_t* idx, uint32_t dn, uint32_t* s_meta,
                              uint32_t* s_flag) {
  uint64_t cur = pos;
  int64_t v = -(int64_t)skip;
  uint32_t lo = 0;
  while (lo < count) {
    if (threadIdx.x < 64) {
      bool bad = false;
      const uint32_t nr = wave_walk(src, cur, v, count, w, MODE == 0, runs, RUNCAP, s_first, bad);
      if (threadIdx.x == 0) {
        s_meta[0] = nr;
        s_meta[1] = (bad || nr == 0) ? 1u : 0u;
        s_meta[2] = (uint32_t)(v < (int64_t)count ? v : (int64_t)count);
      }
    }
    __syncthreads();
    if (s_meta[1]) return false;
    const uint32_t nr = s_meta[0], hi = s_meta[2];
    if (MODE == 0) expand_levels(src, runs, s_first, lo, hi, s_valid);
    else expand_indices(src, runs, nr, s_first, lo, hi, w, dn, idx, s_flag);
    // wave 0 keeps cur / v in registers for the next batch
    lo = hi;
    __syncthreads();
  }
  return true;
}

// ---------------------------------------------------------------------------
// per-tile phases
// ---------------------------------------------------------------------------
struct TileCtx {
  ColScan cs;
  TileDev td;
  PageDev pg;
  Streams st;
  uint32_t t;
  uint32_t nrows;
  int64_t out0;
  bool has_next;   // next tile belongs to the same page
  TileDev next;
};

__device__ __forceinline__ void load_tile(TileCtx& c, const ColScan* cols, const PageDev* pages, const TileDev* tiles,
                                          const SegTable& seg, const uint8_t* file, uint8_t* ws) {
  uint32_t csi, t;
  find_segment(seg, blockIdx.x, csi, t);
  c.cs = cols[csi];
  c.t = t;
  c.td = tiles[t];
  c.pg = pages[c.td.page];
  c.nrows = (uint32_t)min((int64_t)TR, (int64_t)c.pg.num_values - c.td.row0);
  c.out0 = c.pg.row0 + c.td.row0 - c.cs.row_base;
  c.st = page_streams(c.pg, c.cs, file, ws);
  const uint32_t ntiles = (uint32_t)(((int64_t)c.pg.num_values + TR - 1) / TR);
  c.has_next = t + 1 < c.pg.tile_begin + ntiles;
  if (c.has_next) c.next = tiles[t + 1];
}

// Decodes the tile's definition levels into s_valid and writes the output
// validity words; returns false on error (recorded).
__device__ bool tile_levels(const TileCtx& c, uint8_t* s_stage, Run* runs, uint32_t* s_first, uint32_t* s_valid,
                            uint32_t* s_meta, uint32_t* s_flag, uint32_t* err) {
  const Streams& st = c.st;
  const uint64_t a0 = st.doff + c.td.def_pos;
  uint64_t a1 = st.dend;
  if (c.has_next) a1 = min(a1, st.doff + (uint64_t)c.next.def_pos + 16 + ((uint64_t)c.next.def_skip + 7) / 8);
  uint64_t origin;
  uint32_t len;
  const bool staged = stage(s_stage, STAGE_DEF, st.dbase, a0, a1, origin, len);
  __syncthreads();
  bool ok;
  if (staged) {
    LSrc src{s_stage, len};
    ok = decode_hybrid<0>(src, a0 - origin, c.td.def_skip, c.nrows, 1, runs, s_first, s_valid, nullptr, 0, s_meta, s_flag);
  } else {
    GSrc src{st.dbase, a0, st.dend - a0};
    ok = decode_hybrid<0>(src, 0, c.td.def_skip, c.nrows, 1, runs, s_first, s_valid, nullptr, 0, s_meta, s_flag);
  }
  if (!ok) {
    if (threadIdx.x == 0) set_err(err, ERR_LEVELS, c.td.page);
    return false;
  }
  // output bits [out0, out0 + nrows) <- tile bits [0, nrows)
  if (c.cs.validity) {
    const int64_t out0 = c.out0;
    const int64_t w_first = out0 >> 5;
    const int64_t w_last = (out0 + c.nrows - 1) >> 5;
    uint32_t* vout = reinterpret_cast<uint32_t*>(c.cs.validity);
    for (int64_t W = w_first + threadIdx.x; W <= w_last; W += WG) {
      const int64_t b0 = W * 32 - out0;
      uint32_t word;
      if (b0 >= 0) {
        const uint32_t tw = (uint32_t)(b0 >> 5), sh = (uint32_t)(b0 & 31);
        const uint32_t lo = s_valid[tw];
        const uint32_t hi2 = (tw + 1 < NWORDS) ? s_valid[tw + 1] : 0u;
        word = sh ? ((lo >> sh) | (hi2 << (32 - sh))) : lo;
      } else {
        word = s_valid[0] << (uint32_t)(-b0);
      }
      const int64_t lo_b = b0 < 0 ? -b0 : 0;
      const int64_t hi_b = (int64_t)c.nrows - b0 < 32 ? (int64_t)c.nrows - b0 : 32;
      const uint32_t mask = (hi_b >= 32 ? 0xffffffffu : ((1u << hi_b) - 1)) & (0xffffffffu << lo_b);
      word &= mask;
      if (mask == 0xffffffffu) vout[W] = word;
      else if (word) atomicOr(&vout[W], word);
    }
  }
  return true;
}

// exclusive popcount prefix over the tile's validity words (wave 0)
__device__ __forceinline__ void tile_rank_prefix(const uint32_t* s_valid, uint32_t* s_pre, uint32_t nrows) {
  if (threadIdx.x < 64) {
    const uint32_t nw = (nrows + 31) / 32;
    const uint32_t j = threadIdx.x;
    const uint32_t c = j < nw ? __popc(s_valid[j]) : 0;
    const uint32_t inc = wave_incl_scan_u32(c);
    if (j < nw) s_pre[j] = inc - c;
  }
  __syncthreads();
}

__device__ __forceinline__ bool row_valid(const uint32_t* s_valid, uint32_t r) { return (s_valid[r >> 5] >> (r & 31)) & 1u; }
__device__ __forceinline__ uint32_t row_rank(const uint32_t* s_valid, const uint32_t* s_pre, uint32_t r) {
  return s_pre[r >> 5] + __popc(s_valid[r >> 5] & ((1u << (r & 31)) - 1u));
}

// Decodes the tile's dictionary indices (values [0, nn)) into idx; false on
// error (recorded).
__device__ bool tile_indices(const TileCtx& c, uint32_t dn, uint8_t* s_stage, Run* runs, uint32_t* s_first, uint32_t* idx,
                             uint32_t* s_meta, uint32_t* s_flag, uint32_t* err) {
  const Streams& st = c.st;
  const uint32_t w = c.pg.enc_w;
  const uint64_t a0 = st.voff + c.td.val_pos;
  uint64_t a1 = st.vend;
  if (c.has_next && c.next.k0 < c.pg.nonnull)
    a1 = min(a1, st.voff + (uint64_t)c.next.val_pos + 16 + ((uint64_t)c.next.val_skip * w + 7) / 8);
  uint64_t origin;
  uint32_t len;
  if (threadIdx.x == 0) *s_flag = 0;
  const bool staged = stage(s_stage, STAGE_VAL, st.vbase, a0, a1, origin, len);
  __syncthreads();
  bool ok;
  if (staged) {
    LSrc src{s_stage, len};
    ok = decode_hybrid<1>(src, a0 - origin, c.td.val_skip, c.td.nn, w, runs, s_first, nullptr, idx, dn, s_meta, s_flag);
  } else {
    GSrc src{st.vbase, a0, st.vend - a0};
    ok = decode_hybrid<1>(src, 0, c.td.val_skip, c.td.nn, w, runs, s_first, nullptr, idx, dn, s_meta, s_flag);
  }
  if (!ok) {
    if (threadIdx.x == 0) set_err(err, ERR_VALUES, c.td.page);
    return false;
  }
  if (*s_flag) {
    if (threadIdx.x == 0) set_err(err, ERR_DICT_INDEX, c.td.page);
    return false;
  }
  return true;
}

// DELTA_BINARY_PACKED: thread 0 walks the tile's blocks (headers and
// miniblock widths) over the source into LDS.
template <class Src>
__device__ bool delta_blocks(const Src& src, uint64_t pos, const TileCtx& c, bool is32, DBlock* blk, uint32_t* s_meta) {
  if (threadIdx.x == 0) {
    bool bad = false;
    uint32_t nb = 0;
    const uint64_t B = c.pg.enc_w, M = c.pg.enc_m;
    const TileDev& td = c.td;
    if (td.nn > 0 && (uint64_t)td.k0 + td.nn > 1) {
      const uint64_t per = B / M;
      const uint64_t first = td.k0 == 0 ? 1 : td.k0;
      const uint64_t dlo = first - 1;
      const uint64_t dhi = (uint64_t)td.k0 + td.nn - 1;
      const uint64_t total = c.pg.nonnull;
      uint64_t bidx = dlo / B;
      int64_t rel = -(int64_t)td.val_skip;
      uint64_t q = pos;
      const uint32_t maxw = is32 ? 32 : 64;
      while ((uint64_t)((int64_t)dlo + rel) < dhi) {
        if (nb == DBLK_CAP) { bad = true; break; }
        DBlock& D = blk[nb];
        D.dfirst = (int32_t)rel;
        // zigzag ULEB128 min delta
        uint64_t u = 0;
        int s = 0;
        for (;;) {
          const uint32_t b = src.byte(q++);
          if (s < 64) u |= (uint64_t)(b & 0x7f) << s;
          s += 7;
          if (!(b & 0x80) || s > 70) break;
        }
        D.min_delta = unzz(u);
        const uint64_t left = total - 1 - bidx * B;
        const uint64_t used = left < B ? left : B;
        const uint64_t used_mb = (used + per - 1) / per;
        uint64_t bits = 0;
        for (uint64_t m = 0; m < M; ++m) {
          uint32_t w = m < used_mb ? src.byte(q + m) : 0;
          if (w > maxw) { bad = true; w = 0; }
          D.w[m] = (uint8_t)w;
          D.woff[m] = (uint32_t)bits;
          bits += per * w;
        }
        D.nmb = (uint32_t)M;
        q += M;
        D.bit0 = q * 8;
        q += bits / 8;
        rel += (int64_t)B;
        ++bidx;
        ++nb;
      }
    }
    s_meta[1] = bad ? 1u : 0u;
    s_meta[0] = nb;
  }
  __syncthreads();
  return s_meta[1] == 0;
}

// D_k of tile value j: the stream's first value for global value 0, else
// min_delta + packed bits of its miniblock.
template <class Src>
__device__ __forceinline__ uint64_t delta_term(const Src& src, const DBlock* blk, const TileCtx& c, uint32_t j) {
  const uint64_t k = (uint64_t)c.td.k0 + j;
  if (k == 0) return (uint64_t)c.pg.delta_first;
  const uint64_t B = c.pg.enc_w, M = c.pg.enc_m;
  const uint64_t first = c.td.k0 == 0 ? 1 : c.td.k0;
  const uint64_t drel = (k - 1) - (first - 1) + c.td.val_skip;
  const uint64_t bi = drel / B;
  const uint64_t o = drel - bi * B;
  const uint64_t per = B / M;
  const DBlock& D = blk[bi];
  const uint32_t m = (uint32_t)(o / per), i = (uint32_t)(o - (uint64_t)m * per);
  const uint32_t w = D.w[m];
  return (uint64_t)D.min_delta + src.bits(D.bit0 + D.woff[m] + (uint64_t)i * w, w);
}

// Sum (wrapping) of the tile's DELTA terms, or the terms themselves with a
// carry: out_vals[j] = carry + D_0 + ... + D_j.  Returns false on error.
template <bool VALUES>
__device__ bool tile_delta(const TileCtx& c, uint64_t carry, uint8_t* s_stage, DBlock* blk, uint64_t* out_vals,
                           uint64_t* s_tmp, uint32_t* s_meta, uint64_t* sum_out, uint32_t* err) {
  const Streams& st = c.st;
  const bool is32 = c.cs.type == T_INT32;
  const uint64_t a0 = st.voff + c.td.val_pos;
  uint64_t a1 = st.vend;
  if (c.has_next && c.next.k0 < c.pg.nonnull && c.next.val_skip == 0) a1 = min(a1, st.voff + (uint64_t)c.next.val_pos + 16);
  else if (c.has_next && c.next.k0 < c.pg.nonnull)
    a1 = min(a1, st.voff + (uint64_t)c.next.val_pos + 16 + c.pg.enc_m + (uint64_t)c.pg.enc_w * (is32 ? 4 : 8));
  uint64_t origin;
  uint32_t len;
  const bool staged = stage(s_stage, STAGE_VAL, st.vbase, a0, a1, origin, len);
  __syncthreads();
  constexpr int PER = TR / WG;
  uint64_t loc[PER];
  uint64_t acc = 0;
  bool ok;
  if (staged) {
    LSrc src{s_stage, len};
    ok = delta_blocks(src, a0 - origin, c, is32, blk, s_meta);
    if (ok) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t j = threadIdx.x * PER + q;
        acc += j < c.td.nn ? delta_term(src, blk, c, j) : 0;
        loc[q] = acc;
      }
    }
  } else {
    GSrc src{st.vbase, a0, st.vend - a0};
    ok = delta_blocks(src, 0, c, is32, blk, s_meta);
    if (ok) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t j = threadIdx.x * PER + q;
        acc += j < c.td.nn ? delta_term(src, blk, c, j) : 0;
        loc[q] = acc;
      }
    }
  }
  if (!ok) {
    if (threadIdx.x == 0) set_err(err, ERR_DELTA, c.td.page);
    return false;
  }
  uint64_t tot;
  const uint64_t ex = wg_excl_scan_u64(acc, s_tmp, &tot);
  if (VALUES) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t j = threadIdx.x * PER + q;
      if (j < c.td.nn) out_vals[j] = carry + ex + loc[q];
    }
  }
  *sum_out = tot;
  return true;
}

// ---------------------------------------------------------------------------
// k_snappy: one wave per compressed page
// ---------------------------------------------------------------------------

// Copies n bytes dst[i] = src[i] with the lanes of one wave (no overlap).
__device__ __forceinline__ void wave_copy(uint8_t* dst, const uint8_t* src, uint64_t n) {
  const int lane = threadIdx.x & 63;
  for (uint64_t i = lane; i < n; i += 64) dst[i] = src[i];
}

__global__ __launch_bounds__(WG) void k_snappy(const uint8_t* file, const PageDev* pages, const ColScan* cols,
                                               SegTable seg, uint8_t* ws, uint32_t* err) {
  const uint32_t gw = (blockIdx.x * WG + threadIdx.x) >> 6;
  int k = 0;
  for (int j = 1; j < seg.n; ++j) if (seg.s[j].wg0 <= gw) k = j;
  const uint32_t csi = seg.s[k].cs;
  const uint32_t p = seg.s[k].t0 + (gw - seg.s[k].wg0);
  if (p >= seg.s[k].t1) return;
  const ColScan cs = cols[csi];
  const PageDev pg = pages[p];
  if (pg.scratch_len == 0) return;
  uint64_t src_off = pg.payload, src_len = pg.comp_size;
  if (pg.kind == PAGE_DATA_V2) { src_off += (uint64_t)pg.rep_len + (uint64_t)pg.def_len; src_len -= (uint64_t)pg.rep_len + (uint64_t)pg.def_len; }
  const uint8_t* src = file + src_off;
  uint8_t* dst = ws + cs.ws_scratch + (pg.scratch_off - cs.scratch_base);
  volatile uint8_t* vdst = dst;
  const uint64_t total = pg.scratch_len;
  uint64_t pos = 0, op = 0;
  bool bad = false;
  // stream length
  {
    uint64_t v = 0;
    int s = 0;
    for (;;) {
      if (pos >= src_len || s > 28) { bad = true; break; }
      uint32_t b = src[pos++];
      v |= (uint64_t)(b & 0x7f) << s;
      if (!(b & 0x80)) break;
      s += 7;
    }
    if (!bad && v != total) bad = true;
  }
  while (!bad && pos < src_len) {
    const uint32_t t = src[pos++];
    uint64_t len, off = 0;
    if ((t & 3) == 0) {
      uint64_t l = t >> 2;
      if (l >= 60) {
        const uint32_t nb = (uint32_t)l - 59;
        if (pos + nb > src_len) { bad = true; break; }
        l = 0;
        for (uint32_t k = 0; k < nb; ++k) l |= (uint64_t)src[pos + k] << (8 * k);
        pos += nb;
      }
      len = l + 1;
      if (len > src_len - pos || len > total - op) { bad = true; break; }
      wave_copy(dst + op, src + pos, len);
      pos += len;
      op += len;
      continue;
    }
    if ((t & 3) == 1) {
      if (pos + 1 > src_len) { bad = true; break; }
      len = 4 + ((t >> 2) & 7);
      off = ((uint64_t)(t >> 5) << 8) | src[pos];
      pos += 1;
    } else if ((t & 3) == 2) {
      if (pos + 2 > src_len) { bad = true; break; }
      len = (t >> 2) + 1;
      off = (uint64_t)src[pos] | ((uint64_t)src[pos + 1] << 8);
      pos += 2;
    } else {
      if (pos + 4 > src_len) { bad = true; break; }
      len = (t >> 2) + 1;
      off = (uint64_t)src[pos] | ((uint64_t)src[pos + 1] << 8) | ((uint64_t)src[pos + 2] << 16) | ((uint64_t)src[pos + 3] << 24);
      pos += 4;
    }
    if (off == 0 || off > op || len > total - op) { bad = true; break; }
    // make this wave's earlier stores visible to its own L1-bypassing reads
    __builtin_amdgcn_s_waitcnt(0);
    __threadfence_block();
    const int lane = threadIdx.x & 63;
    for (uint64_t i = lane; i < len; i += 64) {
      // source byte op + i - off, repeating with period `off` when overlapping
      const uint64_t s = off >= len ? op + i - off : op - off + (i % off);
      vdst[op + i] = vdst[s];
    }
    op += len;
  }
  if (!bad && op != total) bad = true;
  if (bad && (threadIdx.x & 63) == 0) set_err(err, ERR_SNAPPY, p);
}

// ---------------------------------------------------------------------------
// k_prep: validity words shared by two tiles are cleared before any tile
// ORs into them; REQUIRED columns with a validity buffer get all ones.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_prep(const ColScan* cols, const PageDev* pages, const TileDev* tiles, SegTable seg) {
  const uint32_t gid = blockIdx.x * WG + threadIdx.x;  // one thread per tile
  int k = 0;
  for (int j = 1; j < seg.n; ++j) if (seg.s[j].wg0 <= gid) k = j;
  const uint32_t t = seg.s[k].t0 + (gid - seg.s[k].wg0);
  if (t >= seg.s[k].t1) return;
  const ColScan cs = cols[seg.s[k].cs];
  if (!cs.validity) return;
  const TileDev td = tiles[t];
  const PageDev pg = pages[td.page];
  const uint32_t nrows = (uint32_t)min((int64_t)TILE_ROWS, (int64_t)pg.num_values - td.row0);
  const int64_t r0 = pg.row0 + td.row0 - cs.row_base;
  uint32_t* v = reinterpret_cast<uint32_t*>(cs.validity);
  if (cs.optional) {
    if (r0 & 31) v[r0 >> 5] = 0;
    if ((r0 + nrows) & 31) v[(r0 + nrows) >> 5] = 0;
  } else {
    // REQUIRED: every word whose first row lies in this tile is written
    // whole (ones for rows < rows, zeros past the end)
    for (int64_t W = (r0 + 31) >> 5; W * 32 < r0 + (int64_t)nrows; ++W) {
      const int64_t left = cs.rows - W * 32;
      v[W] = left >= 32 ? 0xffffffffu : ((1u << left) - 1);
    }
  }
}

// ---------------------------------------------------------------------------
// k_dict: dictionary pages of the scanned chunks -> workspace dictionaries.
// grid: (dictionary slots, chunks of entries)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_dict(const uint8_t* file, uint8_t* ws, const ColScan* cols, int ncols,
                                             const PageDev* pages, DictSlot* slots, const uint32_t* strck, uint32_t* err) {
  const uint32_t si = blockIdx.x;
  const uint32_t part = blockIdx.y;
  DictSlot sl = slots[si];
  if (sl.page == ~0u) return;
  // the column owning this slot
  int c = 0;
  for (int j = 1; j < ncols; ++j) if (cols[j].dict_slot0 <= si) c = j;
  const ColScan cs = cols[c];
  const PageDev pg = pages[sl.page];
  const uint8_t* body;
  uint64_t boff;
  if (pg.flags & 2) { body = ws + cs.ws_scratch; boff = pg.val_off - cs.scratch_base; }
  else { body = file; boff = pg.val_off; }
  if (part == 0 && threadIdx.x == 0) { slots[si].body = body; slots[si].body_off = boff; }
  const uint32_t n = sl.n;
  if (cs.type == T_BYTE_ARRAY) {
    // one thread per checkpoint (STR_CK entries): (pos, len) pairs relative to the body
    uint32_t* pairs = reinterpret_cast<uint32_t*>(ws + sl.ws_entries);
    const uint32_t nck = (n + STR_CK - 1) / STR_CK;
    const uint32_t ck = part * WG + threadIdx.x;
    if (ck >= nck) return;
    uint64_t q = strck[pg.strck_begin + ck];
    for (uint32_t j = 0; j < STR_CK; ++j) {
      const uint32_t e = ck * STR_CK + j;
      if (e >= n) break;
      if ((uint64_t)pg.val_len - q < 4) { set_err(err, ERR_STRING, sl.page); return; }
      const uint32_t l = ld_u32(body, boff + q);
      q += 4;
      if (l > (uint64_t)pg.val_len - q) { set_err(err, ERR_STRING, sl.page); return; }
      pairs[2 * e] = (uint32_t)q;
      pairs[2 * e + 1] = l;
      q += l;
    }
  } else {
    const uint32_t w = cs.width;
    for (uint32_t e = part * 8192 + threadIdx.x; e < n && e < (part + 1) * 8192; e += WG) {
      if (w == 4) reinterpret_cast<uint32_t*>(ws + sl.ws_entries)[e] = ld_u32(body, boff + (uint64_t)e * 4);
      else reinterpret_cast<uint64_t*>(ws + sl.ws_entries)[e] = ld_u64(body, boff + (uint64_t)e * 8);
    }
  }
}

// ---------------------------------------------------------------------------
// k_tile_scan: exclusive prefix over each listed column's tile auxiliaries
// (one workgroup per column); string columns also get offsets[rows] and the
// capacity check.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_tile_scan(uint8_t* ws, const ColScan* cols, const int32_t* which, uint32_t* err) {
  __shared__ uint64_t s_tmp[WG / 64];
  const ColScan cs = cols[which[blockIdx.x]];
  uint64_t* aux = reinterpret_cast<uint64_t*>(ws + cs.ws_tile_aux);
  const uint32_t n = cs.tile_end - cs.tile_begin;
  uint64_t carry = 0;
  for (uint32_t b = 0; b < n; b += WG) {
    const uint32_t i = b + threadIdx.x;
    const uint64_t v = i < n ? aux[i] : 0;
    uint64_t tot;
    const uint64_t ex = wg_excl_scan_u64(v, s_tmp, &tot);
    if (i < n) aux[i] = carry + ex;
    carry += tot;
  }
  if (cs.type == T_BYTE_ARRAY && threadIdx.x == 0) {
    if (cs.offsets) cs.offsets[cs.rows] = (int64_t)carry;
    if (carry > cs.chars_capacity) set_err(err, ERR_CAPACITY, (uint32_t)cs.col);
    // slot past the last tile: total (read by pq_plan)
    aux[n] = carry;
  }
}

// ---------------------------------------------------------------------------
// k_prepass: per-tile auxiliaries (DELTA sums, string byte counts)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_prepass(const uint8_t* file, uint8_t* ws, const ColScan* cols, const PageDev* pages,
                                                const TileDev* tiles, const DictSlot* slots, SegTable seg, uint32_t* err) {
  __shared__ __align__(16) uint8_t s_stage[STAGE_VAL];
  __shared__ Run s_runs[RUNCAP];
  __shared__ uint32_t s_first[NWORDS];
  __shared__ __align__(16) uint64_t s_pairs[TR];
  __shared__ DBlock s_blk[DBLK_CAP];
  __shared__ uint64_t s_tmp[NWAVES];
  __shared__ uint32_t s_meta[4];
  __shared__ uint32_t s_flag;
  TileCtx c;
  load_tile(c, cols, pages, tiles, seg, file, ws);
  uint64_t* aux = reinterpret_cast<uint64_t*>(ws + c.cs.ws_tile_aux) + (c.t - c.cs.tile_begin);
  if (c.cs.type != T_BYTE_ARRAY) {  // DELTA tile sum
    uint64_t sum;
    if (!tile_delta<false>(c, 0, s_stage, s_blk, nullptr, s_tmp, s_meta, &sum, err)) return;
    if (threadIdx.x == 0) *aux = sum;
    return;
  }
  if (c.pg.encoding == E_PLAIN) {
    if (threadIdx.x == 0) *aux = (uint64_t)c.td.val_skip - c.td.val_pos - 4ull * c.td.nn;
    return;
  }
  const uint32_t rg = c.pg.chunk % (uint32_t)c.cs.nrg;
  const DictSlot sl = slots[c.cs.dict_slot0 + (rg - (uint32_t)c.cs.rg_begin)];
  if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, c.td.page); return; }
  if (c.td.nn == 0) { if (threadIdx.x == 0) *aux = 0; return; }
  const uint32_t* pairs = reinterpret_cast<const uint32_t*>(ws + sl.ws_entries);
  uint32_t* idx = reinterpret_cast<uint32_t*>(s_pairs);
  if (!tile_indices(c, sl.n, s_stage, s_runs, s_first, idx, s_meta, &s_flag, err)) return;
  __syncthreads();
  uint64_t acc = 0;
  for (uint32_t i = threadIdx.x; i < c.td.nn; i += WG) acc += pairs[2 * idx[i] + 1];
  uint64_t tot;
  wg_excl_scan_u64(acc, s_tmp, &tot);
  if (threadIdx.x == 0) *aux = tot;
}

// ---------------------------------------------------------------------------
// k_decode_fixed: INT32 / INT64 / DOUBLE tiles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_decode_fixed(const uint8_t* file, uint8_t* ws, const ColScan* cols,
                                                     const PageDev* pages, const TileDev* tiles, const DictSlot* slots,
                                                     SegTable seg, uint32_t* err) {
  __shared__ __align__(16) uint8_t s_stage[STAGE_VAL];
  __shared__ Run s_runs[RUNCAP];
  __shared__ uint32_t s_valid[NWORDS];
  __shared__ uint32_t s_pre[NWORDS];
  __shared__ uint32_t s_first[NWORDS];
  __shared__ __align__(16) uint64_t s_vals[TR];
  __shared__ DBlock s_blk[DBLK_CAP];
  __shared__ uint64_t s_tmp[NWAVES];
  __shared__ uint32_t s_meta[4];
  __shared__ uint32_t s_flag;

  TileCtx c;
  load_tile(c, cols, pages, tiles, seg, file, ws);
  const bool opt = c.cs.optional;
  const int width = c.cs.width;
  const uint32_t nrows = c.nrows;
  if (opt) {
    for (uint32_t j = threadIdx.x; j < NWORDS; j += WG) s_valid[j] = 0;
    if (!tile_levels(c, s_stage, s_runs, s_first, s_valid, s_meta, &s_flag, err)) return;
    tile_rank_prefix(s_valid, s_pre, nrows);
  }
  const int enc = c.pg.encoding;
  const int64_t out0 = c.out0;

  if (enc == E_PLAIN) {
    const Streams& st = c.st;
    for (uint32_t r = threadIdx.x; r < nrows; r += WG) {
      const bool v = !opt || row_valid(s_valid, r);
      const uint64_t k = (uint64_t)c.td.k0 + (opt ? row_rank(s_valid, s_pre, r) : r);
      if (width == 4) {
        const uint32_t x = v ? ld_u32(st.vbase, st.voff + k * 4) : 0u;
        reinterpret_cast<uint32_t*>(c.cs.values)[out0 + r] = x;
      } else {
        const uint64_t x = v ? ld_u64(st.vbase, st.voff + k * 8) : 0ull;
        reinterpret_cast<uint64_t*>(c.cs.values)[out0 + r] = x;
      }
    }
    return;
  }

  if (enc == E_PLAIN_DICT || enc == E_RLE_DICT) {
    const uint32_t rg = c.pg.chunk % (uint32_t)c.cs.nrg;
    const DictSlot sl = slots[c.cs.dict_slot0 + (rg - (uint32_t)c.cs.rg_begin)];
    if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, c.td.page); return; }
    uint32_t* idx = reinterpret_cast<uint32_t*>(s_vals);
    if (c.td.nn > 0) {
      if (!tile_indices(c, sl.n, s_stage, s_runs, s_first, idx, s_meta, &s_flag, err)) return;
      __syncthreads();
    }
    const uint8_t* ent = ws + sl.ws_entries;
    for (uint32_t r = threadIdx.x; r < nrows; r += WG) {
      const bool v = !opt || row_valid(s_valid, r);
      const uint32_t k = opt ? row_rank(s_valid, s_pre, r) : r;
      if (width == 4) {
        const uint32_t x = v ? reinterpret_cast<const uint32_t*>(ent)[idx[k]] : 0u;
        reinterpret_cast<uint32_t*>(c.cs.values)[out0 + r] = x;
      } else {
        const uint64_t x = v ? reinterpret_cast<const uint64_t*>(ent)[idx[k]] : 0ull;
        reinterpret_cast<uint64_t*>(c.cs.values)[out0 + r] = x;
      }
    }
    return;
  }

  if (enc == E_DELTA) {
    const uint64_t* aux = reinterpret_cast<const uint64_t*>(ws + c.cs.ws_tile_aux);
    const uint64_t carry = aux[c.t - c.cs.tile_begin] - aux[c.pg.tile_begin - c.cs.tile_begin];
    uint64_t sum;
    if (!tile_delta<true>(c, carry, s_stage, s_blk, s_vals, s_tmp, s_meta, &sum, err)) return;
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < nrows; r += WG) {
      const bool v = !opt || row_valid(s_valid, r);
      const uint32_t k = opt ? row_rank(s_valid, s_pre, r) : r;
      const uint64_t x = v ? s_vals[k] : 0ull;
      if (width == 4) reinterpret_cast<uint32_t*>(c.cs.values)[out0 + r] = (uint32_t)x;
      else reinterpret_cast<uint64_t*>(c.cs.values)[out0 + r] = x;
    }
    return;
  }
  if (threadIdx.x == 0) set_err(err, ERR_UNSUPPORTED, c.td.page);
}

// ---------------------------------------------------------------------------
// k_decode_str: BYTE_ARRAY tiles -> offsets and chars
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_decode_str(const uint8_t* file, uint8_t* ws, const ColScan* cols,
                                                   const PageDev* pages, const TileDev* tiles, const DictSlot* slots,
                                                   const uint32_t* strck, SegTable seg, uint32_t* err) {
  __shared__ __align__(16) uint8_t s_stage[STAGE_VAL];
  __shared__ Run s_runs[RUNCAP];
  __shared__ uint32_t s_valid[NWORDS];
  __shared__ uint32_t s_pre[NWORDS];
  __shared__ uint32_t s_first[NWORDS];
  __shared__ __align__(16) uint64_t s_vals[TR];  // per value: pos | len << 32
  __shared__ uint32_t s_idx[TR];
  __shared__ uint64_t s_tmp[NWAVES];
  __shared__ uint32_t s_meta[4];
  __shared__ uint32_t s_flag;

  TileCtx c;
  load_tile(c, cols, pages, tiles, seg, file, ws);
  const bool opt = c.cs.optional;
  const uint32_t nrows = c.nrows;
  if (opt) {
    for (uint32_t j = threadIdx.x; j < NWORDS; j += WG) s_valid[j] = 0;
    if (!tile_levels(c, s_stage, s_runs, s_first, s_valid, s_meta, &s_flag, err)) return;
    tile_rank_prefix(s_valid, s_pre, nrows);
  }
  if (threadIdx.x == 0) s_flag = 0;
  __syncthreads();

  // ---- (pos, len) of the tile's values; sources are (aligned base, offset) ----
  const uint8_t* sbase;
  uint64_t soff;
  if (c.pg.encoding == E_PLAIN) {
    sbase = c.st.vbase;
    soff = c.st.voff;
    const TileDev& td = c.td;
    const uint32_t ck_lo = td.k0 / STR_CK;
    const uint32_t ck_hi = td.nn ? (td.k0 + td.nn - 1) / STR_CK : ck_lo;
    for (uint32_t ck = ck_lo + threadIdx.x; td.nn && ck <= ck_hi; ck += WG) {
      uint64_t q = strck[c.pg.strck_begin + ck];
      for (uint32_t j = 0; j < STR_CK; ++j) {
        const uint32_t k = ck * STR_CK + j;
        if (k >= td.k0 + td.nn) break;
        if ((uint64_t)c.pg.val_len - q < 4) { s_flag = 1; break; }
        const uint32_t l = ld_u32(c.st.vbase, c.st.voff + q);
        q += 4;
        if (l > (uint64_t)c.pg.val_len - q) { s_flag = 1; break; }
        if (k >= td.k0) s_vals[k - td.k0] = q | ((uint64_t)l << 32);
        q += l;
      }
    }
    __syncthreads();
    if (s_flag) { if (threadIdx.x == 0) set_err(err, ERR_STRING, c.td.page); return; }
  } else {
    const uint32_t rg = c.pg.chunk % (uint32_t)c.cs.nrg;
    const DictSlot sl = slots[c.cs.dict_slot0 + (rg - (uint32_t)c.cs.rg_begin)];
    if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, c.td.page); return; }
    sbase = sl.body;
    soff = sl.body_off;
    if (c.td.nn > 0) {
      if (!tile_indices(c, sl.n, s_stage, s_runs, s_first, s_idx, s_meta, &s_flag, err)) return;
      __syncthreads();
      const uint32_t* pairs = reinterpret_cast<const uint32_t*>(ws + sl.ws_entries);
      for (uint32_t i = threadIdx.x; i < c.td.nn; i += WG) {
        const uint32_t x = s_idx[i];
        s_vals[i] = (uint64_t)pairs[2 * x] | ((uint64_t)pairs[2 * x + 1] << 32);
      }
      __syncthreads();
    }
  }

  // ---- offsets: exclusive scan of row lengths; thread j owns rows [8j, 8j+8) ----
  const uint64_t* aux = reinterpret_cast<const uint64_t*>(ws + c.cs.ws_tile_aux);
  const uint64_t base = aux[c.t - c.cs.tile_begin];
  constexpr int PER = TR / WG;
  uint32_t lens[PER];
  uint64_t acc = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t r = threadIdx.x * PER + q;
    uint32_t l = 0;
    if (r < nrows && (!opt || row_valid(s_valid, r))) l = (uint32_t)(s_vals[opt ? row_rank(s_valid, s_pre, r) : r] >> 32);
    lens[q] = l;
    acc += l;
  }
  uint64_t tot;
  uint64_t run = wg_excl_scan_u64(acc, s_tmp, &tot);
  const bool fits = base + tot <= c.cs.chars_capacity && tot < 0xffffffffull;
  uint32_t* s_off = reinterpret_cast<uint32_t*>(s_stage);  // rows+1 relative offsets (stage is free now)
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t r = threadIdx.x * PER + q;
    if (r < nrows) {
      if (c.cs.offsets) c.cs.offsets[c.out0 + r] = (int64_t)(base + run);
      s_off[r] = (uint32_t)run;
    }
    run += lens[q];
  }
  if (threadIdx.x == 0) s_off[nrows] = (uint32_t)tot;
  __syncthreads();
  if (!fits || !c.cs.chars || tot == 0) return;

  // ---- chars: one wave per 64-row group writes its output range dword by dword ----
  uint8_t* chars = c.cs.chars;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t ngroups = (nrows + 63) / 64;
  for (uint32_t g = wave; g < ngroups; g += NWAVES) {
    const uint32_t r0 = g * 64, r1 = min(r0 + 64, nrows);
    const uint32_t A = s_off[r0], Bq = s_off[r1];
    if (A == Bq) continue;
    const uint64_t d0 = (base + A) >> 2, d1 = (base + Bq + 3) >> 2;
    for (uint64_t d = d0 + lane; d < d1; d += 64) {
      const uint64_t q0a = max(d * 4, base + A), q1a = min(d * 4 + 4, base + Bq);
      const uint32_t q0 = (uint32_t)(q0a - base), q1 = (uint32_t)(q1a - base);
      // last row of the group whose range starts at or before q0
      uint32_t lo = r0, hi = r1 - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= q0) lo = mid; else hi = mid - 1;
      }
      uint32_t row = lo;
      if (q1 - q0 == 4 && s_off[row + 1] >= q1) {
        const uint32_t pos = (uint32_t)s_vals[opt ? row_rank(s_valid, s_pre, row) : row];
        const uint32_t x = ld_u32(sbase, soff + pos + (q0 - s_off[row]));
        *reinterpret_cast<uint32_t*>(chars + d * 4) = x;
      } else {
        for (uint32_t q = q0; q < q1; ++q) {
          while (s_off[row + 1] <= q) ++row;
          const uint32_t pos = (uint32_t)s_vals[opt ? row_rank(s_valid, s_pre, row) : row];
          const uint32_t x = ld_u32(sbase, soff + pos + (q - s_off[row])) & 0xffu;
          chars[base + q] = (uint8_t)x;
        }
      }
    }
  }
}

}  // namespace pqk
