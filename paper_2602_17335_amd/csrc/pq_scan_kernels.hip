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
// 256-thread workgroup, entered through the tile index built at open.  A
// tile issues every global load it needs up front: the byte ranges of its
// level and value streams are copied into LDS with coalesced 16-byte loads.
// One wave then walks the level stream's run headers while another walks the
// value stream's (or a lane walks the DELTA block headers): each lane parses
// the header that would start at its byte, and the real chain is followed
// through those 64 candidates with readlane.  All threads then expand runs,
// compute ranks, and write the outputs with coalesced stores.
#include <hip/hip_runtime.h>

#include "pq_device.hpp"
#include "pq_internal.h"

namespace pqk {

constexpr int WG = 256;
constexpr int NWAVES = WG / 64;
constexpr int TR = TILE_ROWS;        // rows per tile
constexpr int PER = TR / WG;         // rows (or values) per thread
constexpr int NWORDS = TR / 32;      // validity words per tile
constexpr int DRUNCAP = 128;         // level runs per batch
constexpr int VRUNCAP = 64;          // index runs per batch
constexpr int DSTAGE = 1024;         // staged level-stream bytes
constexpr int VSTAGE = TR * 8 + 256; // staged value-stream bytes
constexpr int DBLK_CAP = TR / 128 + 2;
constexpr int DMINI_MAX = 16;
constexpr int GROUP_CHARS = 3072;    // per-wave LDS bytes for one 64-row group of strings

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
// byte sources: a staged copy of a stream range in LDS (LSrc), or the range
// in global memory when it does not fit the LDS buffer (GSrc).  Positions are
// relative to the start of the copy (LSrc) or to `origin` (GSrc).  They are
// separate types so that LDS reads compile to ds_read and global reads to
// global_load.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) const uint8_t lds_u8;
typedef __attribute__((address_space(3))) const uint32_t lds_u32;
typedef __attribute__((address_space(1))) const uint8_t glb_u8;
typedef __attribute__((address_space(1))) const uint32_t glb_u32;

template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

struct LSrc {
  lds_u8* p;     // 16-byte aligned LDS buffer
  uint32_t len;  // staged bytes (multiple of 16)
  __device__ __forceinline__ uint32_t byte(uint64_t i) const { return i < len ? (uint32_t)p[i] : 0u; }
  __device__ __forceinline__ uint32_t dword_at(uint64_t dw) const {
    return dw < (len >> 2) ? reinterpret_cast<lds_u32*>(p)[dw] : 0u;
  }
  __device__ __forceinline__ uint64_t bits(uint64_t bit, uint32_t w) const {
    if (w == 0) return 0;
    const uint64_t dw = bit >> 5;
    const uint32_t sh = (uint32_t)(bit & 31);
    uint64_t v = ((uint64_t)dword_at(dw) | ((uint64_t)dword_at(dw + 1) << 32)) >> sh;
    if (sh + w > 64) v |= (uint64_t)dword_at(dw + 2) << (64 - sh);
    return w == 64 ? v : (v & ((1ull << w) - 1));
  }
  __device__ __forceinline__ uint64_t size() const { return len; }
  __device__ __forceinline__ uint32_t u32(uint64_t pos) const { return (uint32_t)bits(pos * 8, 32); }
  __device__ __forceinline__ uint64_t u64(uint64_t pos) const { return bits(pos * 8, 64); }
};

struct GSrc {
  glb_u8* base;     // 16-byte aligned global base
  uint64_t origin;  // absolute offset of position 0
  uint64_t len;
  __device__ __forceinline__ uint32_t byte(uint64_t i) const { return i < len ? (uint32_t)base[origin + i] : 0u; }
  __device__ __forceinline__ uint64_t bits(uint64_t bit, uint32_t w) const {
    if (w == 0) return 0;
    const uint64_t b = origin * 8 + bit;
    const uint64_t dw = b >> 5;
    const uint32_t sh = (uint32_t)(b & 31);
    glb_u32* q = reinterpret_cast<glb_u32*>(base) + dw;
    uint64_t v = ((uint64_t)q[0] | ((uint64_t)q[1] << 32)) >> sh;
    if (sh + w > 64) v |= (uint64_t)q[2] << (64 - sh);
    return w == 64 ? v : (v & ((1ull << w) - 1));
  }
  __device__ __forceinline__ uint64_t size() const { return len; }
  __device__ __forceinline__ uint32_t u32(uint64_t pos) const { return (uint32_t)bits(pos * 8, 32); }
  __device__ __forceinline__ uint64_t u64(uint64_t pos) const { return bits(pos * 8, 64); }
};

// A staged stream: bytes [a0, a1) of `base` copied into LDS from the 16-byte
// boundary at or below a0 when they fit `cap`, else left in global memory.
struct Staged {
  bool in_lds;
  LSrc l;
  GSrc g;
  uint64_t pos0;  // position of a0 in the source
};

// Issues the loads of a stage (no barrier); threads tid, tid+stride, ...
// copy 16 bytes each.
__device__ __forceinline__ Staged stage(uint8_t* lds, uint32_t cap, const uint8_t* base, uint64_t a0, uint64_t a1,
                                        uint32_t tid = threadIdx.x, uint32_t stride = WG) {
  Staged s;
  if (a1 < a0) a1 = a0;
  const uint64_t org = a0 & ~15ull;
  const uint64_t n16 = (a1 - org + 15) >> 4;
  s.l.p = (lds_u8*)lds;
  s.l.len = 0;
  s.g.base = (glb_u8*)base;
  s.g.origin = a0;
  s.g.len = a1 - a0;
  if (n16 * 16 <= cap) {
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const __attribute__((address_space(1))) v4u* src = reinterpret_cast<const __attribute__((address_space(1))) v4u*>(
        (glb_u8*)base + org);
    __attribute__((address_space(3))) v4u* dst = reinterpret_cast<__attribute__((address_space(3))) v4u*>(
        (__attribute__((address_space(3))) uint8_t*)lds);
    for (uint32_t i = tid; i < (uint32_t)n16; i += stride) dst[i] = src[i];
    s.in_lds = true;
    s.l.len = (uint32_t)(n16 * 16);
    s.pos0 = a0 - org;
  } else {
    s.in_lds = false;
    s.pos0 = 0;
  }
  return s;
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
struct WalkState {
  uint64_t cur;   // position of the next run header
  int64_t v;      // tile-relative first value of the run at `cur`
  uint32_t nr;    // runs recorded in the current batch
  uint32_t lo;    // first value of the current batch
  uint32_t hi;    // values covered by the current batch (clamped to count)
  uint32_t bad;
};

// Follows the chain of run headers from st.cur until `count` values are
// covered or `cap` runs are recorded.  Executed by all lanes of one wave.
// Each lane parses the header that would start at cur + lane.  When the run
// at cur spans the whole 64-byte window it is taken alone; otherwise the
// chain through the 64 candidates is resolved in parallel: successor tables
// J_k (2^k steps) are built by pointer doubling with ds_bpermute, and each
// lane finds, by binary lifting from the chain start, the last chain element
// at or before itself (it is on the chain iff that is itself).  Chain lanes
// prefix-sum their value counts, and the runs the tile needs are written to
// the run table together with the first-run marks of the 32-value words they
// cover.  Lane 0 updates `st`.
template <class Src>
__device__ void walk_batch(const Src& src, WalkState* st, uint32_t count, uint32_t w, bool levels, Run* runs,
                           uint32_t cap, uint32_t* s_first) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint64_t cur = st->cur;
  int64_t v = st->v;
  const uint32_t lo = (uint32_t)max((int64_t)0, v);
  uint32_t nr = 0;
  bool bad = false;
  while (v < (int64_t)count && nr < cap) {
    const uint64_t p = cur + (uint64_t)lane;
    uint32_t b[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) b[k] = src.byte(p + k);
    uint32_t hl = 0;
    bool ok = false;
#pragma unroll
    for (int k = 4; k >= 0; --k)
      if (!(b[k] & 0x80)) { hl = k + 1; ok = true; }
    uint64_t h = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if ((uint32_t)k < hl) h |= (uint64_t)(b[k] & 0x7f) << (7 * k);
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
      for (int k = 0; k < 4; ++k) {
        uint32_t x = 0;
#pragma unroll
        for (int j = 1; j < 9; ++j)
          if ((uint32_t)j == hl + k) x = b[j];
        if ((uint32_t)k < plen) val |= x << (8 * k);
      }
      if (levels && val > 1) ok = false;
    }
    if (cnt > 0x7fffffffull || plen > 0x7fffffffull || p + hl > src.size()) ok = false;
    const uint32_t adv = max(1u, (uint32_t)min(hl + plen, (uint64_t)0x7fffffffull));
    const uint64_t ps = p + hl;  // payload start

    uint32_t adv0 = (uint32_t)__builtin_amdgcn_readlane((int)adv, 0);
    uint64_t mask;    // chain lanes the tile needs (recorded)
    uint64_t incl;    // inclusive prefix of counts over chain lanes
    uint64_t cm;
    bool onchain;
    if (adv0 >= 64) {
      onchain = lane == 0;
    } else {
      // successor tables and binary lifting (64 = outside the window)
      const uint32_t nxt = min((uint32_t)lane + adv, 64u);
      uint32_t J[6];
      J[0] = nxt;
#pragma unroll
      for (int k = 1; k < 6; ++k) {
        const uint32_t prev = J[k - 1];
        const uint32_t nn2 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(min(prev, 63u) << 2), (int)prev);
        J[k] = prev < 64 ? nn2 : 64u;
      }
      uint32_t pos = 0;
#pragma unroll
      for (int k = 5; k >= 0; --k) {
        const uint32_t nx = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(pos << 2), (int)J[k]);
        if (nx <= (uint32_t)lane) pos = nx;
      }
      onchain = pos == (uint32_t)lane;
    }
    cm = onchain ? cnt : 0ull;
    incl = wave_incl_scan_u64(cm);
    const int64_t vs = v + (int64_t)(incl - cm);
    const bool needed = onchain && vs < (int64_t)count && cnt > 0;
    const uint64_t need_mask = __ballot(needed);
    const uint32_t rk = (uint32_t)__popcll(need_mask & lt_mask);
    const bool keep = needed && nr + rk < cap;
    // the part of each kept run the tile needs must lie inside the source
    const uint64_t need = keep ? min(cnt, (uint64_t)((int64_t)count - vs)) : 0ull;
    const uint64_t nb = isbp ? (need * w + 7) / 8 : (uint64_t)(w + 7) / 8;
    const bool badl = (onchain && !ok && vs < (int64_t)count) || (keep && ps + nb > src.size());
    if (__ballot(badl)) { bad = true; break; }
    mask = __ballot(keep);
    if (keep) {
      const uint32_t kk = nr + rk;
      Run R;
      R.vstart = (int32_t)vs;
      R.nbp = (uint32_t)cnt | (isbp ? 0x80000000u : 0u);
      R.pay = isbp ? ps * 8 : (uint64_t)val;
      runs[kk] = R;
      int64_t j = vs <= 0 ? 0 : (vs + 31) >> 5;
      for (; j < NWORDS && j * 32 < vs + (int64_t)cnt; ++j) s_first[j] = kk;
    }
    const uint32_t nkept = (uint32_t)__popcll(mask);
    if (nr + (uint32_t)__popcll(need_mask) > cap) {
      // table full: continue at the first needed run that was not recorded
      const uint64_t fm = __ballot(needed && nr + rk == cap);
      const int f = __builtin_ctzll(fm);
      const uint64_t inc_f = ((uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)incl, f)) |
                             ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(incl >> 32), f) << 32);
      const uint64_t cm_f = ((uint64_t)__builtin_amdgcn_readlane((int)(uint32_t)cm, f)) |
                            ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(cm >> 32), f) << 32);
      v = v + (int64_t)(inc_f - cm_f);
      cur = cur + (uint64_t)f;
      nr = cap;
      break;
    }
    nr += nkept;
    // advance past the window: the last chain lane's successor
    const uint64_t em = __ballot(onchain && (adv0 >= 64 || (uint32_t)lane + adv >= 64));
    const int e = em ? 63 - __builtin_clzll(em) : 0;
    const uint64_t inc_e = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)incl, e)) |
                           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(incl >> 32), e) << 32);
    v += (int64_t)inc_e;
    cur += (uint64_t)e + (uint32_t)__builtin_amdgcn_readlane((int)adv, e);
  }
  if (lane == 0) {
    st->cur = cur;
    st->v = v;
    st->nr = nr;
    st->lo = lo;
    st->hi = (uint32_t)(v < (int64_t)count ? v : (int64_t)count);
    st->bad = (bad || (nr == 0 && lo < count)) ? 1u : 0u;
  }
}

// Expands the definition levels of rows [lo, hi) into the LDS validity words
// (one thread per 32-row word).
template <class Src>
__device__ void expand_levels(const Src& src, const Run* runs, const uint32_t* s_first, uint32_t lo, uint32_t hi,
                              uint32_t* s_valid, uint32_t tid, uint32_t stride) {
  const uint32_t w0 = lo >> 5, w1 = (hi + 31) >> 5;
  for (uint32_t j = w0 + tid; j < w1; j += stride) {
    uint32_t r = max(j * 32, lo);
    const uint32_t re = min(j * 32 + 32, hi);
    uint32_t k = (j * 32 < lo) ? 0u : s_first[j];
    uint32_t word = 0;
    while (r < re) {
      const Run R = runs[k];
      const uint32_t n = R.nbp & 0x7fffffffu;
      const uint32_t e = (uint32_t)min((int64_t)re, (int64_t)R.vstart + n);
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

// Decodes values [lo, hi) of an index stream (bit width w) into idx[];
// flags indices >= dn.
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

// ---------------------------------------------------------------------------
// DELTA_BINARY_PACKED: one lane walks the tile's blocks into LDS
// ---------------------------------------------------------------------------
template <class Src>
__device__ void delta_blocks(const Src& src, uint64_t pos, const PageDev& pg, const TileDev& td, bool is32, DBlock* blk,
                             uint32_t* s_dmeta) {
  bool bad = false;
  uint32_t nb = 0;
  const uint64_t B = pg.enc_w, M = pg.enc_m;
  if (td.nn > 0 && (uint64_t)td.k0 + td.nn > 1) {
    const uint64_t per = B / M;
    const uint64_t first = td.k0 == 0 ? 1 : td.k0;
    const uint64_t dlo = first - 1;
    const uint64_t dhi = (uint64_t)td.k0 + td.nn - 1;
    const uint64_t total = pg.nonnull;
    uint64_t bidx = dlo / B;
    int64_t rel = -(int64_t)td.val_skip;
    uint64_t q = pos;
    const uint32_t maxw = is32 ? 32 : 64;
    while ((uint64_t)((int64_t)dlo + rel) < dhi) {
      if (nb == DBLK_CAP || q >= src.size()) { bad = true; break; }
      DBlock& D = blk[nb];
      D.dfirst = (int32_t)rel;
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
  s_dmeta[1] = bad ? 1u : 0u;
  s_dmeta[0] = nb;
}

// D_j of tile value j: the stream's first value for global value 0, else
// min_delta + packed bits of its miniblock.
template <class Src>
__device__ __forceinline__ uint64_t delta_term(const Src& src, const DBlock* blk, const PageDev& pg, const TileDev& td,
                                               uint32_t j) {
  const uint64_t k = (uint64_t)td.k0 + j;
  if (k == 0) return (uint64_t)pg.delta_first;
  const uint64_t B = pg.enc_w, M = pg.enc_m;
  const uint64_t first = td.k0 == 0 ? 1 : td.k0;
  const uint64_t drel = (k - 1) - (first - 1) + td.val_skip;
  const uint64_t bi = drel / B;
  const uint64_t o = drel - bi * B;
  const uint64_t per = B / M;
  const DBlock& D = blk[bi];
  const uint32_t m = (uint32_t)(o / per), i = (uint32_t)(o - (uint64_t)m * per);
  const uint32_t w = D.w[m];
  return (uint64_t)D.min_delta + src.bits(D.bit0 + D.woff[m] + (uint64_t)i * w, w);
}

// ---------------------------------------------------------------------------
// per-tile context and stream ranges
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
  c.t = t;
  c.td = tiles[t];
  c.next = tiles[t + 1 < seg.s[seg.n - 1].t1 ? t + 1 : t];
  c.cs = cols[csi];
  c.pg = pages[c.td.page];
  c.nrows = (uint32_t)min((int64_t)TR, (int64_t)c.pg.num_values - c.td.row0);
  c.out0 = c.pg.row0 + c.td.row0 - c.cs.row_base;
  c.st = page_streams(c.pg, c.cs, file, ws);
  c.has_next = c.next.page == c.td.page && c.next.row0 > c.td.row0;
}

// level-stream byte range a tile needs
__device__ __forceinline__ void level_range(const TileCtx& c, uint64_t& a0, uint64_t& a1) {
  a0 = c.st.doff + c.td.def_pos;
  a1 = c.st.dend;
  if (c.has_next) a1 = min(a1, c.st.doff + (uint64_t)c.next.def_pos + 16 + ((uint64_t)c.next.def_skip + 7) / 8);
}

// value-stream byte range a tile needs
__device__ __forceinline__ void value_range(const TileCtx& c, uint64_t& a0, uint64_t& a1) {
  const int enc = c.pg.encoding;
  const bool nextvals = c.has_next && c.next.k0 < c.pg.nonnull;
  if (enc == E_PLAIN && c.cs.type == T_BYTE_ARRAY) {  // strings: located through checkpoints
    a0 = a1 = c.st.voff;
    return;
  }
  if (enc == E_PLAIN) {
    const uint64_t w = c.cs.width;
    a0 = c.st.voff + (uint64_t)c.td.k0 * w;
    a1 = a0 + (uint64_t)c.td.nn * w;
  } else if (enc == E_DELTA) {
    a0 = c.st.voff + c.td.val_pos;
    a1 = c.st.vend;
    if (nextvals) {
      const uint64_t more = c.next.val_skip ? 16 + c.pg.enc_m + (uint64_t)c.pg.enc_w * (c.cs.type == T_INT32 ? 4 : 8) : 16;
      a1 = min(a1, c.st.voff + (uint64_t)c.next.val_pos + more);
    }
  } else {  // dictionary indices
    a0 = c.st.voff + c.td.val_pos;
    a1 = c.st.vend;
    if (nextvals) a1 = min(a1, c.st.voff + (uint64_t)c.next.val_pos + 16 + ((uint64_t)c.next.val_skip * c.pg.enc_w + 7) / 8);
  }
  if (c.td.nn == 0) a1 = a0;
}

// Writes the tile's validity words into the output bitmap.
__device__ __forceinline__ void write_validity(const TileCtx& c, const uint32_t* s_valid, uint32_t tid,
                                               uint32_t stride) {
  if (!c.cs.validity) return;
  const int64_t out0 = c.out0;
  const int64_t w_first = out0 >> 5;
  const int64_t w_last = (out0 + c.nrows - 1) >> 5;
  __attribute__((address_space(1))) uint32_t* vout = gptr(reinterpret_cast<uint32_t*>(c.cs.validity));
  for (int64_t W = w_first + tid; W <= w_last; W += stride) {
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
    if (mask == 0xffffffffu) __builtin_nontemporal_store(word, &vout[W]);
    else if (word) atomicOr(reinterpret_cast<uint32_t*>(c.cs.validity) + W, word);
  }
}

// exclusive popcount prefix over the tile's validity words (wave 0)
__device__ __forceinline__ void tile_rank_prefix(const uint32_t* s_valid, uint32_t* s_pre, uint32_t nrows) {
  if (threadIdx.x < 64) {
    const uint32_t nw = (nrows + 31) / 32;
    const uint32_t j = threadIdx.x;
    const uint32_t cnt = j < nw ? __popc(s_valid[j]) : 0;
    const uint32_t inc = wave_incl_scan_u32(cnt);
    if (j < nw) s_pre[j] = inc - cnt;
  }
}

__device__ __forceinline__ bool row_valid(const uint32_t* s_valid, uint32_t r) { return (s_valid[r >> 5] >> (r & 31)) & 1u; }
__device__ __forceinline__ uint32_t row_rank(const uint32_t* s_valid, const uint32_t* s_pre, uint32_t r) {
  return s_pre[r >> 5] + __popc(s_valid[r >> 5] & ((1u << (r & 31)) - 1u));
}

// Shared state of the front half of a decode tile (levels, values).
struct TileShared {
  uint32_t valid[NWORDS];
  uint32_t pre[NWORDS];
  uint32_t vfirst[NWORDS];
  WalkState vst;
  uint32_t dmeta[2];
  uint32_t flag;
  uint64_t tmp[NWAVES];
  Run vruns[VRUNCAP];
  __attribute__((aligned(16))) uint8_t vstage[VSTAGE];
};

// Loads the tile's validity words (written by k_levels) from the output
// bitmap: tile bit i = output bit out0 + i.
__device__ __forceinline__ void load_validity(const TileCtx& c, uint32_t* s_valid) {
  if (threadIdx.x < NWORDS) {
    const uint32_t j = threadIdx.x;
    uint32_t word = 0;
    if (j * 32 < c.nrows) {
      const int64_t b = c.out0 + (int64_t)j * 32;
      const __attribute__((address_space(1))) uint32_t* v = gptr(reinterpret_cast<const uint32_t*>(c.cs.validity));
      const int64_t W = b >> 5;
      const uint32_t sh = (uint32_t)(b & 31);
      const int64_t nw = (c.cs.rows + 31) >> 5;
      const uint32_t lo = v[W];
      const uint32_t hi = (sh && W + 1 < nw) ? v[W + 1] : 0u;
      word = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
      const uint32_t rem = c.nrows - j * 32;
      if (rem < 32) word &= (1u << rem) - 1;
    }
    s_valid[j] = word;
  }
}

// Front half of a decode tile: loads the validity words (k_levels wrote
// them) and stages the value stream; then one wave walks the dictionary
// index runs (or one lane the DELTA blocks) while the ranks are computed,
// and all threads expand the indices into idx.  Returns false on error
// (recorded).  `vs` describes the staged value stream.
#define PQ_WITH_SRC(S, CALL) \
  do {                       \
    if ((S).in_lds) {        \
      const LSrc& src_ = (S).l; \
      CALL;                  \
    } else {                 \
      const GSrc& src_ = (S).g; \
      CALL;                  \
    }                        \
  } while (0)

__device__ bool tile_front(const TileCtx& c, TileShared& sh, uint32_t dict_n, uint32_t* idx, DBlock* blk, Staged& vs,
                           uint32_t* err) {
  const bool opt = c.cs.optional;
  const int enc = c.pg.encoding;
  const bool is_dict = enc == E_PLAIN_DICT || enc == E_RLE_DICT;
  const bool is_delta = enc == E_DELTA;
  uint64_t v0, v1;
  value_range(c, v0, v1);
  vs = stage(sh.vstage, VSTAGE, c.st.vbase, v0, v1);
  if (opt) load_validity(c, sh.valid);
  if (threadIdx.x == 0) {
    sh.flag = 0;
    sh.vst.cur = vs.pos0; sh.vst.v = -(int64_t)c.td.val_skip; sh.vst.bad = 0;
    sh.dmeta[0] = 0; sh.dmeta[1] = 0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  // the walking wave rotates with the workgroup so walkers spread over the SIMDs
  const int wval = (blockIdx.x + 1) & 3, wdelta = (blockIdx.x + 2) & 3, wrank = blockIdx.x & 3;
  const bool idx_walk = is_dict && c.td.nn > 0;
  const uint32_t w = c.pg.enc_w;
  if (wave == wval && idx_walk) PQ_WITH_SRC(vs, walk_batch(src_, &sh.vst, c.td.nn, w, false, sh.vruns, VRUNCAP, sh.vfirst));
  if ((int)threadIdx.x == wdelta * 64 && is_delta)
    PQ_WITH_SRC(vs, delta_blocks(src_, vs.pos0, c.pg, c.td, c.cs.type == T_INT32, blk, sh.dmeta));
  if (wave == wrank && opt) {
    // exclusive popcount prefix over the validity words
    const uint32_t j = threadIdx.x & 63;
    const uint32_t cnt = j < NWORDS ? __popc(sh.valid[j]) : 0;
    const uint32_t inc = wave_incl_scan_u32(cnt);
    if (j < NWORDS) sh.pre[j] = inc - cnt;
  }
  __syncthreads();
  if (idx_walk) {
    for (;;) {
      if (sh.vst.bad) { if (threadIdx.x == 0) set_err(err, ERR_VALUES, c.td.page); return false; }
      PQ_WITH_SRC(vs, expand_indices(src_, sh.vruns, sh.vst.nr, sh.vfirst, sh.vst.lo, sh.vst.hi, w, dict_n, idx, &sh.flag));
      if (sh.vst.hi >= c.td.nn) break;
      __syncthreads();
      if (wave == wval) PQ_WITH_SRC(vs, walk_batch(src_, &sh.vst, c.td.nn, w, false, sh.vruns, VRUNCAP, sh.vfirst));
      __syncthreads();
    }
  }
  if (is_delta && sh.dmeta[1]) { if (threadIdx.x == 0) set_err(err, ERR_DELTA, c.td.page); return false; }
  __syncthreads();
  if (sh.flag) { if (threadIdx.x == 0) set_err(err, ERR_DICT_INDEX, c.td.page); return false; }
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
// k_levels: definition levels -> output validity, one wave per tile
// ---------------------------------------------------------------------------
struct LevelShared {
  uint32_t valid[NWORDS];
  uint32_t first[NWORDS];
  WalkState st;
  Run runs[DRUNCAP];
  __attribute__((aligned(16))) uint8_t stage[DSTAGE];
};

// Orders this wave's LDS accesses (no other wave takes part).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(WG) void k_levels(const uint8_t* __restrict__ file, uint8_t* __restrict__ ws,
                                               const ColScan* __restrict__ cols, const PageDev* __restrict__ pages,
                                               const TileDev* __restrict__ tiles, SegTable seg,
                                               uint32_t* __restrict__ err) {
  __shared__ LevelShared lsh[NWAVES];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  LevelShared& sh = lsh[wave];
  const uint32_t unit = blockIdx.x * NWAVES + wave;
  int k = 0;
  for (int j = 1; j < seg.n; ++j)
    if (seg.s[j].wg0 <= unit) k = j;
  const uint32_t t = seg.s[k].t0 + (unit - seg.s[k].wg0);
  if (t >= seg.s[k].t1) return;  // the whole wave leaves
  TileCtx c;
  c.t = t;
  c.td = tiles[t];
  c.next = tiles[t + 1 < seg.s[seg.n - 1].t1 ? t + 1 : t];
  c.cs = cols[seg.s[k].cs];
  c.pg = pages[c.td.page];
  c.nrows = (uint32_t)min((int64_t)TR, (int64_t)c.pg.num_values - c.td.row0);
  c.out0 = c.pg.row0 + c.td.row0 - c.cs.row_base;
  c.st = page_streams(c.pg, c.cs, file, ws);
  c.has_next = c.next.page == c.td.page && c.next.row0 > c.td.row0;
  uint64_t d0, d1;
  level_range(c, d0, d1);
  const Staged ds = stage(sh.stage, DSTAGE, c.st.dbase, d0, d1, lane, 64);
  for (uint32_t j = lane; j < NWORDS; j += 64) sh.valid[j] = 0;
  if (lane == 0) { sh.st.cur = ds.pos0; sh.st.v = -(int64_t)c.td.def_skip; sh.st.bad = 0; }
  wave_sync();
  for (;;) {
    PQ_WITH_SRC(ds, walk_batch(src_, &sh.st, c.nrows, 1, true, sh.runs, DRUNCAP, sh.first));
    wave_sync();
    if (sh.st.bad) { if (lane == 0) set_err(err, ERR_LEVELS, c.td.page); return; }
    const uint32_t lo = sh.st.lo, hi = sh.st.hi;
    PQ_WITH_SRC(ds, expand_levels(src_, sh.runs, sh.first, lo, hi, sh.valid, lane, 64));
    wave_sync();
    if (hi >= c.nrows) break;
  }
  write_validity(c, sh.valid, lane, 64);
}

// ---------------------------------------------------------------------------
// k_prepass: per-tile auxiliaries (DELTA sums, string byte counts)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_prepass(const uint8_t* __restrict__ file, uint8_t* __restrict__ ws,
                                                const ColScan* __restrict__ cols, const PageDev* __restrict__ pages,
                                                const TileDev* __restrict__ tiles, const DictSlot* __restrict__ slots,
                                                SegTable seg, uint32_t* __restrict__ err) {
  __shared__ __align__(16) uint8_t s_stage[VSTAGE];
  __shared__ Run s_runs[VRUNCAP];
  __shared__ uint32_t s_first[NWORDS];
  __shared__ uint32_t s_idx[TR];
  __shared__ DBlock s_blk[DBLK_CAP];
  __shared__ uint64_t s_tmp[NWAVES];
  __shared__ WalkState s_st;
  __shared__ uint32_t s_dmeta[2];
  __shared__ uint32_t s_flag;
  TileCtx c;
  load_tile(c, cols, pages, tiles, seg, file, ws);
  __attribute__((address_space(1))) uint64_t* aux =
      reinterpret_cast<__attribute__((address_space(1))) uint64_t*>(gptr(ws + c.cs.ws_tile_aux)) + (c.t - c.cs.tile_begin);
  const bool is_str = c.cs.type == T_BYTE_ARRAY;
  if (is_str && c.pg.encoding == E_PLAIN) {
    if (threadIdx.x == 0) *aux = (uint64_t)c.td.val_skip - c.td.val_pos - 4ull * c.td.nn;
    return;
  }
  if (c.td.nn == 0) { if (threadIdx.x == 0) *aux = 0; return; }
  uint64_t a0, a1;
  value_range(c, a0, a1);
  const Staged vs = stage(s_stage, VSTAGE, c.st.vbase, a0, a1);
  if (threadIdx.x == 0) { s_flag = 0; s_st.cur = vs.pos0; s_st.v = -(int64_t)c.td.val_skip; s_st.bad = 0; }
  __syncthreads();
  uint64_t acc = 0;
  if (!is_str) {  // DELTA tile sum
    if (threadIdx.x == 0) PQ_WITH_SRC(vs, delta_blocks(src_, vs.pos0, c.pg, c.td, c.cs.type == T_INT32, s_blk, s_dmeta));
    __syncthreads();
    if (s_dmeta[1]) { if (threadIdx.x == 0) set_err(err, ERR_DELTA, c.td.page); return; }
    PQ_WITH_SRC(vs, {
      for (int q = 0; q < PER; ++q) {
        const uint32_t j = threadIdx.x * PER + q;
        if (j < c.td.nn) acc += delta_term(src_, s_blk, c.pg, c.td, j);
      }
    });
  } else {  // dictionary strings: sum of entry lengths over the tile's indices
    const uint32_t rg = c.pg.chunk % (uint32_t)c.cs.nrg;
    const DictSlot sl = slots[c.cs.dict_slot0 + (rg - (uint32_t)c.cs.rg_begin)];
    if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, c.td.page); return; }
    for (;;) {
      if (threadIdx.x < 64) PQ_WITH_SRC(vs, walk_batch(src_, &s_st, c.td.nn, c.pg.enc_w, false, s_runs, VRUNCAP, s_first));
      __syncthreads();
      if (s_st.bad) { if (threadIdx.x == 0) set_err(err, ERR_VALUES, c.td.page); return; }
      PQ_WITH_SRC(vs, expand_indices(src_, s_runs, s_st.nr, s_first, s_st.lo, s_st.hi, c.pg.enc_w, sl.n, s_idx, &s_flag));
      if (s_st.hi >= c.td.nn) break;
      __syncthreads();
    }
    __syncthreads();
    if (s_flag) { if (threadIdx.x == 0) set_err(err, ERR_DICT_INDEX, c.td.page); return; }
    glb_u32* pairs = reinterpret_cast<glb_u32*>(gptr(ws + sl.ws_entries));
    uint32_t l[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t i = threadIdx.x + q * WG;
      l[q] = i < c.td.nn ? pairs[2 * s_idx[i] + 1] : 0u;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) acc += l[q];
  }
  uint64_t tot;
  wg_excl_scan_u64(acc, s_tmp, &tot);
  if (threadIdx.x == 0) *aux = tot;
}

// ---------------------------------------------------------------------------
// k_decode_fixed: INT32 / INT64 / DOUBLE tiles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_decode_fixed(const uint8_t* __restrict__ file, uint8_t* __restrict__ ws,
                                                     const ColScan* __restrict__ cols, const PageDev* __restrict__ pages,
                                                     const TileDev* __restrict__ tiles,
                                                     const DictSlot* __restrict__ slots, SegTable seg,
                                                     uint32_t* __restrict__ err) {
  __shared__ TileShared sh;
  __shared__ __align__(16) uint64_t s_vals[TR];
  __shared__ DBlock s_blk[DBLK_CAP];

  TileCtx c;
  load_tile(c, cols, pages, tiles, seg, file, ws);
  const bool opt = c.cs.optional;
  const int width = c.cs.width;
  const int enc = c.pg.encoding;
  const bool is_dict = enc == E_PLAIN_DICT || enc == E_RLE_DICT;
  DictSlot sl;
  sl.page = ~0u;
  sl.n = 0;
  sl.ws_entries = 0;
  if (is_dict) {
    const uint32_t rg = c.pg.chunk % (uint32_t)c.cs.nrg;
    sl = slots[c.cs.dict_slot0 + (rg - (uint32_t)c.cs.rg_begin)];
    if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, c.td.page); return; }
  }
  uint32_t* idx = reinterpret_cast<uint32_t*>(s_vals);
  Staged vs;
  if (!tile_front(c, sh, sl.n, idx, s_blk, vs, err)) return;
  const uint64_t vpos = vs.pos0;
  const uint32_t nrows = c.nrows;
  const int64_t out0 = c.out0;
  __attribute__((address_space(1))) uint32_t* out32 = gptr(reinterpret_cast<uint32_t*>(c.cs.values));
  __attribute__((address_space(1))) uint64_t* out64 = gptr(reinterpret_cast<uint64_t*>(c.cs.values));

  // rows r = threadIdx.x + q*WG: coalesced stores; every load is issued before the stores
  if (enc == E_PLAIN) {
    if (width == 4) {
      uint32_t x[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        const bool v = r < nrows && (!opt || row_valid(sh.valid, r));
        const uint32_t k = opt ? row_rank(sh.valid, sh.pre, r) : r;
        PQ_WITH_SRC(vs, x[q] = v ? src_.u32(vpos + (uint64_t)k * 4) : 0u);
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        if (r < nrows) __builtin_nontemporal_store(x[q], &out32[out0 + r]);
      }
    } else {
      uint64_t x[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        const bool v = r < nrows && (!opt || row_valid(sh.valid, r));
        const uint32_t k = opt ? row_rank(sh.valid, sh.pre, r) : r;
        PQ_WITH_SRC(vs, x[q] = v ? src_.u64(vpos + (uint64_t)k * 8) : 0ull);
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        if (r < nrows) __builtin_nontemporal_store(x[q], &out64[out0 + r]);
      }
    }
    return;
  }

  if (is_dict) {
    glb_u8* ent = gptr(ws + sl.ws_entries);
    if (width == 4) {
      uint32_t x[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        const bool v = r < nrows && (!opt || row_valid(sh.valid, r));
        const uint32_t k = opt ? row_rank(sh.valid, sh.pre, r) : r;
        x[q] = v ? reinterpret_cast<glb_u32*>(ent)[idx[k]] : 0u;
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        if (r < nrows) __builtin_nontemporal_store(x[q], &out32[out0 + r]);
      }
    } else {
      uint64_t x[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        const bool v = r < nrows && (!opt || row_valid(sh.valid, r));
        const uint32_t k = opt ? row_rank(sh.valid, sh.pre, r) : r;
        x[q] = v ? reinterpret_cast<const __attribute__((address_space(1))) uint64_t*>(ent)[idx[k]] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const uint32_t r = threadIdx.x + q * WG;
        if (r < nrows) __builtin_nontemporal_store(x[q], &out64[out0 + r]);
      }
    }
    return;
  }

  if (enc == E_DELTA) {
    const uint64_t* aux = reinterpret_cast<const uint64_t*>(ws + c.cs.ws_tile_aux);
    const uint64_t carry = aux[c.t - c.cs.tile_begin] - aux[c.pg.tile_begin - c.cs.tile_begin];
    // thread j owns values [PER*j, PER*j + PER)
    uint64_t loc[PER];
    uint64_t acc = 0;
#pragma unroll
    PQ_WITH_SRC(vs, {
      for (int q = 0; q < PER; ++q) {
        const uint32_t j = threadIdx.x * PER + q;
        acc += j < c.td.nn ? delta_term(src_, s_blk, c.pg, c.td, j) : 0;
        loc[q] = acc;
      }
    });
    uint64_t tot;
    const uint64_t ex = wg_excl_scan_u64(acc, sh.tmp, &tot);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t j = threadIdx.x * PER + q;
      if (j < c.td.nn) s_vals[j] = carry + ex + loc[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t r = threadIdx.x + q * WG;
      if (r >= nrows) break;
      const bool v = !opt || row_valid(sh.valid, r);
      const uint32_t k = opt ? row_rank(sh.valid, sh.pre, r) : r;
      const uint64_t x = v ? s_vals[k] : 0ull;
      if (width == 4) __builtin_nontemporal_store((uint32_t)x, &out32[out0 + r]);
      else __builtin_nontemporal_store(x, &out64[out0 + r]);
    }
    return;
  }
  if (threadIdx.x == 0) set_err(err, ERR_UNSUPPORTED, c.td.page);
}

// ---------------------------------------------------------------------------
// string copy: one lane copies one string of L bytes from source offset S of a
// 4-byte aligned base to chars offset D, 32 bytes per step: nine aligned
// source dwords are loaded together, realigned with byte funnel shifts, and
// written as aligned dwords (bytes at the string's two ends).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void copy_string(glb_u8* sbase, uint64_t S, __attribute__((address_space(1))) uint8_t* chars,
                                            uint64_t D, uint32_t L) {
  for (uint32_t j0 = 0; j0 < L; j0 += 32) {
    const uint32_t n = min(32u, L - j0);
    const uint64_t s = S + j0, d = D + j0;
    glb_u32* q = reinterpret_cast<glb_u32*>(sbase + (s & ~3ull));
    const uint32_t ss = (uint32_t)(s & 3);
    const uint32_t nsw = (ss + n + 3) >> 2;
    uint32_t w[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) w[k] = (uint32_t)k < nsw ? q[k] : 0u;
    uint32_t rr[9];  // string bytes [4k, 4k+4) of this step
#pragma unroll
    for (int k = 0; k < 9; ++k) rr[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], ss);
    const uint32_t dd = (uint32_t)(d & 3);
    __attribute__((address_space(1))) uint32_t* dw =
        reinterpret_cast<__attribute__((address_space(1))) uint32_t*>(chars + (d & ~3ull));
    const uint32_t ndw = (dd + n + 3) >> 2;
#pragma unroll
    for (int m = 0; m < 10; ++m) {
      if ((uint32_t)m >= ndw) break;
      const uint32_t prev = m == 0 ? 0u : rr[m - 1 < 9 ? m - 1 : 8];
      const uint32_t curw = m < 9 ? rr[m] : 0u;
      const uint32_t word = dd ? __builtin_amdgcn_alignbyte(curw, prev, 4 - dd) : curw;
      // bytes of destination word m that belong to this string: [lo, hi)
      const int lo = m == 0 ? (int)dd : 0;
      const int hi = (int)min(4u, dd + n - 4u * (uint32_t)m);
      if (lo == 0 && hi == 4) {
        __builtin_nontemporal_store(word, &dw[m]);
      } else {
        __attribute__((address_space(1))) uint8_t* b = reinterpret_cast<__attribute__((address_space(1))) uint8_t*>(dw + m);
        for (int k = lo; k < hi; ++k) b[k] = (uint8_t)(word >> (8 * k));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_decode_str: BYTE_ARRAY tiles -> offsets and chars
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_decode_str(const uint8_t* __restrict__ file, uint8_t* __restrict__ ws,
                                                   const ColScan* __restrict__ cols, const PageDev* __restrict__ pages,
                                                   const TileDev* __restrict__ tiles,
                                                   const DictSlot* __restrict__ slots,
                                                   const uint32_t* __restrict__ strck, SegTable seg,
                                                   uint32_t* __restrict__ err) {
  __shared__ TileShared sh;
  __shared__ __align__(16) uint64_t s_vals[TR];  // per value: pos | len << 32
  __shared__ uint32_t s_idx[TR + 1];

  TileCtx c;
  load_tile(c, cols, pages, tiles, seg, file, ws);
  const bool opt = c.cs.optional;
  const uint32_t nrows = c.nrows;
  const bool is_plain = c.pg.encoding == E_PLAIN;
  DictSlot sl;
  sl.page = ~0u;
  sl.n = 0;
  sl.ws_entries = 0;
  sl.body = nullptr;
  sl.body_off = 0;
  if (!is_plain) {
    const uint32_t rg = c.pg.chunk % (uint32_t)c.cs.nrg;
    sl = slots[c.cs.dict_slot0 + (rg - (uint32_t)c.cs.rg_begin)];
    if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, c.td.page); return; }
  }
  Staged vs;
  if (!tile_front(c, sh, sl.n, s_idx, nullptr, vs, err)) return;

  // ---- (pos, len) of the tile's values; source = (aligned base, offset) ----
  const uint8_t* sbase;
  uint64_t soff;
  if (is_plain) {
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
        if ((uint64_t)c.pg.val_len - q < 4) { sh.flag = 1; break; }
        const uint32_t l = ld_u32(c.st.vbase, c.st.voff + q);
        q += 4;
        if (l > (uint64_t)c.pg.val_len - q) { sh.flag = 1; break; }
        if (k >= td.k0) s_vals[k - td.k0] = q | ((uint64_t)l << 32);
        q += l;
      }
    }
    __syncthreads();
    if (sh.flag) { if (threadIdx.x == 0) set_err(err, ERR_STRING, c.td.page); return; }
  } else {
    sbase = sl.body;
    soff = sl.body_off;
    const __attribute__((address_space(1))) uint64_t* pairs =
        reinterpret_cast<const __attribute__((address_space(1))) uint64_t*>(gptr(ws + sl.ws_entries));
    uint64_t pv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t i = threadIdx.x + q * WG;
      pv[q] = i < c.td.nn ? pairs[s_idx[i]] : 0ull;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t i = threadIdx.x + q * WG;
      if (i < c.td.nn) s_vals[i] = pv[q];
    }
    __syncthreads();
  }

  // ---- offsets: exclusive scan of row lengths; thread j owns rows [PER*j, PER*j+PER) ----
  const __attribute__((address_space(1))) uint64_t* aux =
      reinterpret_cast<const __attribute__((address_space(1))) uint64_t*>(gptr(ws + c.cs.ws_tile_aux));
  const uint64_t base = aux[c.t - c.cs.tile_begin];
  uint32_t lens[PER];
  uint64_t acc = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t r = threadIdx.x * PER + q;
    uint32_t l = 0;
    if (r < nrows && (!opt || row_valid(sh.valid, r))) l = (uint32_t)(s_vals[opt ? row_rank(sh.valid, sh.pre, r) : r] >> 32);
    lens[q] = l;
    acc += l;
  }
  uint64_t tot;
  uint64_t run = wg_excl_scan_u64(acc, sh.tmp, &tot);
  if (tot >= 0xffffffffull) { if (threadIdx.x == 0) set_err(err, ERR_UNSUPPORTED, c.td.page); return; }
  const bool fits = base + tot <= c.cs.chars_capacity;
  uint32_t* s_off = s_idx;  // tile-relative row offsets (indices are no longer needed)
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t r = threadIdx.x * PER + q;
    if (r < nrows) {
      if (c.cs.offsets) __builtin_nontemporal_store((int64_t)(base + run), &gptr(c.cs.offsets)[c.out0 + r]);
      s_off[r] = (uint32_t)run;
    }
    run += lens[q];
  }
  if (threadIdx.x == 0) s_off[nrows] = (uint32_t)tot;
  __syncthreads();
  if (!fits || !c.cs.chars) return;
  __attribute__((address_space(1))) uint8_t* chars = gptr(c.cs.chars);
  glb_u8* sb = (glb_u8*)sbase;
  // chars: neighbouring lanes copy neighbouring rows
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t r = threadIdx.x + q * WG;
    if (r >= nrows) break;
    const uint32_t len = s_off[r + 1] - s_off[r];
    if (len) {
      const uint32_t pos = (uint32_t)s_vals[opt ? row_rank(sh.valid, sh.pre, r) : r];
      copy_string(sb, soff + pos, chars, base + s_off[r], len);
    }
  }
}

}  // namespace pqk
