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
// 256-thread workgroup, entered through the tile index built at open.
#include <hip/hip_runtime.h>

#include "pq_device.hpp"
#include "pq_internal.h"

namespace pqk {

constexpr int WG = 256;
constexpr int RUNCAP = 512;
constexpr int DBLK_CAP = 40;
constexpr int DMINI_MAX = 16;

struct Run {
  int32_t vstart;  // first value (tile-relative; negative for a run entered mid-way)
  uint32_t n;
  uint32_t bp;     // 1: bit-packed
  uint32_t pad;
  uint64_t pay;    // bit-packed: absolute bit position of the payload; RLE: the value
};

struct DBlock {
  int32_t dfirst;   // first delta index of the block, relative to the tile's first delta
  uint32_t pad;
  int64_t min_delta;
  uint64_t bit0;    // absolute bit position of miniblock 0's body
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

// exclusive scan of one u64 per thread over the workgroup; returns the
// exclusive prefix, *total receives the sum (wrapping)
__device__ __forceinline__ uint64_t wg_excl_scan_u64(uint64_t v, uint64_t* s_tmp, uint64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = wave_incl_scan_u64(v);
  if (lane == 63) s_tmp[wave] = inc;
  __syncthreads();
  uint64_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < WG / 64; ++k) {
    uint64_t x = s_tmp[k];
    if (k < wave) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// ---------------------------------------------------------------------------
// RLE / bit-packed hybrid decode by one workgroup
// ---------------------------------------------------------------------------
// Decodes values [0, count) of a hybrid stream whose run header at `pos`
// holds the first value after `skip` already-consumed values of that run.
// Thread 0 walks run headers into the LDS run table (up to RUNCAP runs per
// batch); all threads then expand the batch, one value per thread, calling
// emit(i, value, active) with every lane of every wave (active = i valid).
// Returns false on a malformed stream (error already recorded).
template <class Emit>
__device__ bool wg_hybrid(const uint8_t* base, uint64_t pos, uint64_t end, uint32_t skip, uint32_t w, uint32_t count,
                          bool levels, Run* runs, uint32_t* s_meta, uint64_t* s_pos, uint32_t* err, uint32_t where,
                          Emit emit) {
  uint32_t done = 0;
  if (threadIdx.x == 0) { *s_pos = pos; s_meta[2] = skip; }
  __syncthreads();
  while (done < count) {
    if (threadIdx.x == 0) {
      BR r;
      r.init(base);
      uint64_t cur = *s_pos;
      int64_t v = (int64_t)done - (int64_t)s_meta[2];
      uint32_t nr = 0;
      bool bad = false;
      while (v < (int64_t)count && nr < RUNCAP) {
        uint64_t q = cur;
        uint64_t h = br_uleb(r, q, end, bad);
        if (bad) break;
        Run R;
        R.vstart = (int32_t)v;
        R.pad = 0;
        if (h & 1) {
          uint64_t g = h >> 1;
          uint64_t nb = g * w;
          if (g > (1ull << 28) || nb > end - q) { bad = true; break; }
          R.n = (uint32_t)(g * 8);
          R.bp = 1;
          R.pay = q * 8;
          cur = q + nb;
        } else {
          uint64_t n = h >> 1;
          uint32_t vb = (w + 7) / 8;
          if (n > 0x7fffffffull || vb > end - q) { bad = true; break; }
          uint32_t val = 0;
          for (uint32_t j = 0; j < vb; ++j) val |= r.byte(q + j) << (8 * j);
          if (levels && val > 1) { bad = true; break; }
          R.n = (uint32_t)n;
          R.bp = 0;
          R.pay = val;
          cur = q + vb;
        }
        if (R.n) runs[nr++] = R;
        v += R.n;
      }
      if (nr == 0 && !bad) bad = true;  // no progress: stream exhausted
      if (bad) set_err(err, levels ? ERR_LEVELS : ERR_VALUES, where);
      s_meta[0] = nr;
      s_meta[1] = bad ? 1u : 0u;
      s_meta[3] = (uint32_t)(v < (int64_t)count ? v : (int64_t)count);
      s_meta[2] = 0;
      *s_pos = cur;
    }
    __syncthreads();
    if (s_meta[1]) return false;
    const uint32_t nr = s_meta[0];
    const uint32_t hi = s_meta[3];
    for (uint32_t b = done; b < hi; b += WG) {
      const uint32_t i = b + threadIdx.x;
      const bool active = i < hi;
      uint32_t val = 0;
      if (active) {
        int lo = 0, up = (int)nr - 1;
        while (lo < up) {
          int mid = (lo + up + 1) >> 1;
          if (runs[mid].vstart <= (int32_t)i) lo = mid; else up = mid - 1;
        }
        const Run R = runs[lo];
        val = R.bp ? (uint32_t)get_bits(base, R.pay + (uint64_t)((int32_t)i - R.vstart) * w, w) : (uint32_t)R.pay;
      }
      emit(i, val, active, b);
    }
    done = hi;
    __syncthreads();
  }
  return true;
}

// Decodes a tile's definition levels into the LDS bitmap s_valid (tile-row
// bits) and writes them into the output validity bitmap.
__device__ bool tile_levels(const Streams& st, const TileDev& td, uint32_t nrows, int64_t out_row0, uint8_t* validity,
                            uint32_t* s_valid, Run* runs, uint32_t* s_meta, uint64_t* s_pos, uint32_t* err,
                            uint32_t where) {
  for (uint32_t j = threadIdx.x; j < TILE_ROWS / 32; j += WG) s_valid[j] = 0;
  __syncthreads();
  auto emit = [&](uint32_t i, uint32_t v, bool active, uint32_t b) {
    uint64_t m = __ballot(active && v);
    if ((threadIdx.x & 63) == 0 && m) {
      uint32_t i0 = b + (threadIdx.x & ~63u);
      uint32_t w0 = i0 >> 5, sh = i0 & 31;
      atomicOr(&s_valid[w0], (uint32_t)(m << sh));
      uint64_t rest = sh ? (m >> (32 - sh)) : (m >> 32);
      if ((uint32_t)rest) atomicOr(&s_valid[w0 + 1], (uint32_t)rest);
      if (sh && (uint32_t)(rest >> 32)) atomicOr(&s_valid[w0 + 2], (uint32_t)(rest >> 32));
    }
  };
  if (!wg_hybrid(st.dbase, st.doff + td.def_pos, st.dend, td.def_skip, 1, nrows, true, runs, s_meta, s_pos, err, where,
                 emit))
    return false;
  __syncthreads();
  if (validity) {
    // output bits [out_row0, out_row0 + nrows) <- tile bits [0, nrows)
    const int64_t w_first = out_row0 >> 5;
    const int64_t w_last = (out_row0 + nrows - 1) >> 5;
    uint32_t* vout = reinterpret_cast<uint32_t*>(validity);
    for (int64_t W = w_first + threadIdx.x; W <= w_last; W += WG) {
      const int64_t b0 = W * 32 - out_row0;  // tile bit of output bit 0 of word W
      uint32_t word = 0;
      if (b0 >= 0) {
        const uint32_t tw = (uint32_t)(b0 >> 5), sh = (uint32_t)(b0 & 31);
        uint32_t lo = s_valid[tw];
        uint32_t hi2 = (tw + 1 < TILE_ROWS / 32) ? s_valid[tw + 1] : 0u;
        word = sh ? ((lo >> sh) | (hi2 << (32 - sh))) : lo;
      } else {
        word = s_valid[0] << (uint32_t)(-b0);
      }
      // keep only bits that belong to this tile
      const int64_t lo_b = b0 < 0 ? -b0 : 0;                                // first valid bit in word
      const int64_t hi_b = (int64_t)nrows - b0 < 32 ? (int64_t)nrows - b0 : 32;  // one past last
      uint32_t mask = (hi_b >= 32 ? 0xffffffffu : ((1u << hi_b) - 1)) & (0xffffffffu << lo_b);
      word &= mask;
      if (mask == 0xffffffffu) vout[W] = word;
      else if (word) atomicOr(&vout[W], word);
    }
  }
  return true;
}

// exclusive popcount prefix over the tile's validity words
__device__ __forceinline__ void tile_rank_prefix(const uint32_t* s_valid, uint32_t* s_pre, uint32_t nrows) {
  if (threadIdx.x < 64) {
    const uint32_t nw = (nrows + 31) / 32;
    uint32_t carry = 0;
    for (uint32_t b = 0; b < nw; b += 64) {
      uint32_t j = b + threadIdx.x;
      uint32_t c = j < nw ? __popc(s_valid[j]) : 0;
      uint32_t inc = c;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(inc, d, 64);
        if ((int)threadIdx.x >= d) inc += o;
      }
      if (j < nw) s_pre[j] = carry + inc - c;
      carry += __shfl(inc, 63, 64);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ bool row_valid(const uint32_t* s_valid, uint32_t r) { return (s_valid[r >> 5] >> (r & 31)) & 1u; }
__device__ __forceinline__ uint32_t row_rank(const uint32_t* s_valid, const uint32_t* s_pre, uint32_t r) {
  return s_pre[r >> 5] + __popc(s_valid[r >> 5] & ((1u << (r & 31)) - 1u));
}

// ---------------------------------------------------------------------------
// DELTA_BINARY_PACKED: the tile's deltas
// ---------------------------------------------------------------------------
struct DeltaHdr {
  uint64_t B, M, total;
  int64_t first;
  uint64_t blocks_at;  // position after the header
};

// Thread 0 parses the stream header and walks the tile's blocks into LDS.
// dlo/dhi: delta indices [dlo, dhi) the tile needs (delta d links value d to d+1).
__device__ bool delta_walk(const uint8_t* vbase, uint64_t voff, uint64_t vend, const TileDev& td, bool is32,
                           DBlock* blk, uint32_t* s_meta, DeltaHdr* s_hdr, uint32_t* err, uint32_t where) {
  if (threadIdx.x == 0) {
    BR r;
    r.init(vbase);
    bool bad = false;
    uint64_t q = voff;
    DeltaHdr h;
    h.B = br_uleb(r, q, vend, bad);
    h.M = br_uleb(r, q, vend, bad);
    h.total = br_uleb(r, q, vend, bad);
    h.first = unzz(br_uleb(r, q, vend, bad));
    h.blocks_at = q;
    if (bad || h.B == 0 || h.B % 128 || h.M == 0 || h.M > DMINI_MAX || h.B % h.M || (h.B / h.M) % 32) bad = true;
    uint32_t nb = 0;
    if (!bad && td.nn > 0 && (uint64_t)td.k0 + td.nn > 1) {
      const uint64_t per = h.B / h.M;
      const uint64_t first = td.k0 == 0 ? 1 : td.k0;
      const uint64_t dlo = first - 1;
      const uint64_t dhi = (uint64_t)td.k0 + td.nn - 1;
      uint64_t bidx = dlo / h.B;  // global block index
      int64_t rel = -(int64_t)td.val_skip;
      q = voff + td.val_pos;
      const uint32_t maxw = is32 ? 32 : 64;
      while ((uint64_t)((int64_t)dlo + rel) < dhi) {
        if (nb == DBLK_CAP) { bad = true; break; }
        DBlock& B = blk[nb];
        B.dfirst = (int32_t)rel;
        B.min_delta = unzz(br_uleb(r, q, vend, bad));
        if (bad || h.M > vend - q) { bad = true; break; }
        const uint64_t left = h.total - 1 - bidx * h.B;
        const uint64_t used = left < h.B ? left : h.B;
        const uint64_t used_mb = (used + per - 1) / per;
        uint64_t bits = 0;
        for (uint64_t m = 0; m < h.M; ++m) {
          uint32_t w = m < used_mb ? r.byte(q + m) : 0;
          if (w > maxw) { bad = true; break; }
          B.w[m] = (uint8_t)w;
          B.woff[m] = (uint32_t)bits;
          bits += per * w;
        }
        if (bad) break;
        q += h.M;
        B.bit0 = q * 8;
        if (bits / 8 > vend - q) { bad = true; break; }
        q += bits / 8;
        rel += (int64_t)h.B;
        ++bidx;
        ++nb;
      }
    }
    if (bad) set_err(err, ERR_DELTA, where);
    s_meta[1] = bad ? 1u : 0u;
    s_meta[0] = nb;
    *s_hdr = h;
  }
  __syncthreads();
  return s_meta[1] == 0;
}

// Delta contribution D_k of value k of the tile (k relative): the header's
// first value for global value 0, else min_delta + packed bits.
__device__ __forceinline__ uint64_t delta_term(const uint8_t* vbase, const DBlock* blk, const DeltaHdr& h,
                                               const TileDev& td, uint32_t j) {
  const uint64_t k = (uint64_t)td.k0 + j;
  if (k == 0) return (uint64_t)h.first;
  const uint64_t first = td.k0 == 0 ? 1 : td.k0;
  const int64_t drel = (int64_t)(k - 1) - (int64_t)(first - 1) + (int64_t)td.val_skip;  // >= 0
  const uint64_t bi = (uint64_t)drel / h.B;
  const uint64_t o = (uint64_t)drel % h.B;
  const uint64_t per = h.B / h.M;
  const DBlock& B = blk[bi];
  const uint32_t m = (uint32_t)(o / per), i = (uint32_t)(o % per);
  const uint32_t w = B.w[m];
  const uint64_t u = get_bits(vbase, B.bit0 + B.woff[m] + (uint64_t)i * w, w);
  return (uint64_t)B.min_delta + u;
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
  if (part == 0 && threadIdx.x == 0) slots[si].body = body + boff;
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
// k_prepass: per-tile auxiliaries (DELTA sums, string byte counts)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_prepass(const uint8_t* file, uint8_t* ws, const ColScan* cols, const PageDev* pages,
                                                const TileDev* tiles, const DictSlot* slots, SegTable seg, uint32_t* err) {
  __shared__ Run s_runs[RUNCAP];
  __shared__ DBlock s_blk[DBLK_CAP];
  __shared__ uint32_t s_meta[8];
  __shared__ uint64_t s_pos;
  __shared__ DeltaHdr s_hdr;
  __shared__ uint64_t s_tmp[WG / 64];
  __shared__ uint64_t s_acc;
  uint32_t csi, t;
  find_segment(seg, blockIdx.x, csi, t);
  const ColScan cs = cols[csi];
  const TileDev td = tiles[t];
  const PageDev pg = pages[td.page];
  const Streams st = page_streams(pg, cs, file, ws);
  uint64_t* aux = reinterpret_cast<uint64_t*>(ws + cs.ws_tile_aux) + (t - cs.tile_begin);
  if (threadIdx.x == 0) s_acc = 0;
  __syncthreads();
  if (cs.type != T_BYTE_ARRAY) {  // DELTA tile sum
    if (!delta_walk(st.vbase, st.voff, st.vend, td, cs.type == T_INT32, s_blk, s_meta, &s_hdr, err, td.page)) return;
    const DeltaHdr h = s_hdr;
    uint64_t acc = 0;
    for (uint32_t j = threadIdx.x; j < td.nn; j += WG) acc += delta_term(st.vbase, s_blk, h, td, j);
    uint64_t tot;
    wg_excl_scan_u64(acc, s_tmp, &tot);
    if (threadIdx.x == 0) *aux = tot;
    return;
  }
  if (pg.encoding == E_PLAIN) {
    if (threadIdx.x == 0) *aux = (uint64_t)td.val_skip - td.val_pos - 4ull * td.nn;
    return;
  }
  // dictionary strings: sum of entry lengths over the tile's indices
  const uint32_t rg = (pg.chunk % (uint32_t)cs.nrg);
  const DictSlot sl = slots[cs.dict_slot0 + (rg - (uint32_t)cs.rg_begin)];
  if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, td.page); return; }
  if (td.nn == 0) { if (threadIdx.x == 0) *aux = 0; return; }
  const uint32_t w = ld_u32(st.vbase, st.voff) & 0xff;
  const uint32_t* pairs = reinterpret_cast<const uint32_t*>(ws + sl.ws_entries);
  uint64_t acc = 0;
  bool oob = false;
  auto emit = [&](uint32_t i, uint32_t v, bool active, uint32_t) {
    if (!active) return;
    if (v >= sl.n) { oob = true; return; }
    acc += pairs[2 * v + 1];
  };
  if (!wg_hybrid(st.vbase, st.voff + td.val_pos, st.vend, td.val_skip, w, td.nn, false, s_runs, s_meta, &s_pos, err,
                 td.page, emit))
    return;
  if (oob) set_err(err, ERR_DICT_INDEX, td.page);
  uint64_t tot;
  wg_excl_scan_u64(acc, s_tmp, &tot);
  if (threadIdx.x == 0) *aux = tot;
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
// k_decode_fixed: INT32 / INT64 / DOUBLE tiles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_decode_fixed(const uint8_t* file, uint8_t* ws, const ColScan* cols,
                                                     const PageDev* pages, const TileDev* tiles, const DictSlot* slots,
                                                     SegTable seg, uint32_t* err) {
  __shared__ uint32_t s_valid[TILE_ROWS / 32];
  __shared__ uint32_t s_pre[TILE_ROWS / 32];
  __shared__ Run s_runs[RUNCAP];
  __shared__ uint32_t s_meta[8];
  __shared__ uint64_t s_pos;
  __shared__ DeltaHdr s_hdr;
  __shared__ DBlock s_blk[DBLK_CAP];
  __shared__ uint64_t s_tmp[WG / 64];
  __shared__ uint64_t s_vals[TILE_ROWS];
  __shared__ uint32_t s_flag;

  uint32_t csi, t;
  find_segment(seg, blockIdx.x, csi, t);
  const ColScan cs = cols[csi];
  const TileDev td = tiles[t];
  const PageDev pg = pages[td.page];
  const uint32_t nrows = (uint32_t)min((int64_t)TILE_ROWS, (int64_t)pg.num_values - td.row0);
  const int64_t out0 = pg.row0 + td.row0 - cs.row_base;
  const Streams st = page_streams(pg, cs, file, ws);
  const int width = cs.width;

  if (cs.optional) {
    if (!tile_levels(st, td, nrows, out0, cs.validity, s_valid, s_runs, s_meta, &s_pos, err, td.page)) return;
    tile_rank_prefix(s_valid, s_pre, nrows);
  }
  const bool opt = cs.optional;
  const int enc = pg.encoding;

  if (enc == E_PLAIN) {
    for (uint32_t r = threadIdx.x; r < nrows; r += WG) {
      const bool v = !opt || row_valid(s_valid, r);
      const uint64_t k = (uint64_t)td.k0 + (opt ? row_rank(s_valid, s_pre, r) : r);
      if (width == 4) {
        const uint32_t x = v ? ld_u32(st.vbase, st.voff + k * 4) : 0u;
        reinterpret_cast<uint32_t*>(cs.values)[out0 + r] = x;
      } else {
        const uint64_t x = v ? ld_u64(st.vbase, st.voff + k * 8) : 0ull;
        reinterpret_cast<uint64_t*>(cs.values)[out0 + r] = x;
      }
    }
    return;
  }

  if (enc == E_PLAIN_DICT || enc == E_RLE_DICT) {
    const uint32_t rg = pg.chunk % (uint32_t)cs.nrg;
    const DictSlot sl = slots[cs.dict_slot0 + (rg - (uint32_t)cs.rg_begin)];
    if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, td.page); return; }
    if (threadIdx.x == 0) s_flag = 0;
    __syncthreads();
    if (td.nn > 0) {
      const uint32_t w = ld_u32(st.vbase, st.voff) & 0xff;
      uint32_t* idx = reinterpret_cast<uint32_t*>(s_vals);
      const uint32_t dn = sl.n;
      auto emit = [&](uint32_t i, uint32_t v, bool active, uint32_t) {
        if (!active) return;
        if (v >= dn) { s_flag = 1; v = 0; }
        idx[i] = v;
      };
      if (!wg_hybrid(st.vbase, st.voff + td.val_pos, st.vend, td.val_skip, w, td.nn, false, s_runs, s_meta, &s_pos, err,
                     td.page, emit))
        return;
      __syncthreads();
      if (s_flag) { if (threadIdx.x == 0) set_err(err, ERR_DICT_INDEX, td.page); return; }
    }
    const uint32_t* idx = reinterpret_cast<const uint32_t*>(s_vals);
    const uint8_t* ent = ws + sl.ws_entries;
    for (uint32_t r = threadIdx.x; r < nrows; r += WG) {
      const bool v = !opt || row_valid(s_valid, r);
      const uint32_t k = opt ? row_rank(s_valid, s_pre, r) : r;
      if (width == 4) {
        const uint32_t x = v ? reinterpret_cast<const uint32_t*>(ent)[idx[k]] : 0u;
        reinterpret_cast<uint32_t*>(cs.values)[out0 + r] = x;
      } else {
        const uint64_t x = v ? reinterpret_cast<const uint64_t*>(ent)[idx[k]] : 0ull;
        reinterpret_cast<uint64_t*>(cs.values)[out0 + r] = x;
      }
    }
    return;
  }

  if (enc == E_DELTA) {
    if (!delta_walk(st.vbase, st.voff, st.vend, td, cs.type == T_INT32, s_blk, s_meta, &s_hdr, err, td.page)) return;
    const DeltaHdr h = s_hdr;
    // carry = sum of the earlier tiles of this page (exclusive column prefix
    // minus that of the page's first tile)
    const uint64_t* aux = reinterpret_cast<const uint64_t*>(ws + cs.ws_tile_aux);
    const uint64_t carry = aux[t - cs.tile_begin] - aux[pg.tile_begin - cs.tile_begin];
    // thread j handles values [16j, 16j+16)
    constexpr int PER = TILE_ROWS / WG;
    uint64_t loc[PER];
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t j = threadIdx.x * PER + q;
      const uint64_t d = j < td.nn ? delta_term(st.vbase, s_blk, h, td, j) : 0;
      acc += d;
      loc[q] = acc;
    }
    uint64_t tot;
    const uint64_t ex = wg_excl_scan_u64(acc, s_tmp, &tot);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const uint32_t j = threadIdx.x * PER + q;
      if (j < td.nn) s_vals[j] = carry + ex + loc[q];
    }
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < nrows; r += WG) {
      const bool v = !opt || row_valid(s_valid, r);
      const uint32_t k = opt ? row_rank(s_valid, s_pre, r) : r;
      const uint64_t x = v ? s_vals[k] : 0ull;
      if (width == 4) reinterpret_cast<uint32_t*>(cs.values)[out0 + r] = (uint32_t)x;
      else reinterpret_cast<uint64_t*>(cs.values)[out0 + r] = x;
    }
    return;
  }
  if (threadIdx.x == 0) set_err(err, ERR_UNSUPPORTED, td.page);
}

// ---------------------------------------------------------------------------
// k_decode_str: BYTE_ARRAY tiles -> offsets and chars
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_decode_str(const uint8_t* file, uint8_t* ws, const ColScan* cols,
                                                   const PageDev* pages, const TileDev* tiles, const DictSlot* slots,
                                                   const uint32_t* strck, SegTable seg, uint32_t* err) {
  __shared__ uint32_t s_valid[TILE_ROWS / 32];
  __shared__ uint32_t s_pre[TILE_ROWS / 32];
  __shared__ Run s_runs[RUNCAP];
  __shared__ uint32_t s_meta[8];
  __shared__ uint64_t s_pos;
  __shared__ uint64_t s_tmp[WG / 64];
  __shared__ uint64_t s_vals[TILE_ROWS];  // (pos | len << 32) per value
  __shared__ uint32_t s_flag;

  uint32_t csi, t;
  find_segment(seg, blockIdx.x, csi, t);
  const ColScan cs = cols[csi];
  const TileDev td = tiles[t];
  const PageDev pg = pages[td.page];
  const uint32_t nrows = (uint32_t)min((int64_t)TILE_ROWS, (int64_t)pg.num_values - td.row0);
  const int64_t out0 = pg.row0 + td.row0 - cs.row_base;
  const Streams st = page_streams(pg, cs, file, ws);
  const bool opt = cs.optional;

  if (opt) {
    if (!tile_levels(st, td, nrows, out0, cs.validity, s_valid, s_runs, s_meta, &s_pos, err, td.page)) return;
    tile_rank_prefix(s_valid, s_pre, nrows);
  }
  if (threadIdx.x == 0) s_flag = 0;
  __syncthreads();

  // ---- (pos, len) of the tile's values, and the source base ----
  const uint8_t* src;
  uint64_t src_off;
  if (pg.encoding == E_PLAIN) {
    src = st.vbase;
    src_off = st.voff;
    const uint32_t ck_lo = td.k0 / STR_CK;
    const uint32_t ck_hi = td.nn ? (td.k0 + td.nn - 1) / STR_CK : ck_lo;
    for (uint32_t c = ck_lo + threadIdx.x; td.nn && c <= ck_hi; c += WG) {
      uint64_t q = strck[pg.strck_begin + c];
      for (uint32_t j = 0; j < STR_CK; ++j) {
        const uint32_t k = c * STR_CK + j;
        if (k >= td.k0 + td.nn) break;
        if ((uint64_t)pg.val_len - q < 4) { s_flag = 1; break; }
        const uint32_t l = ld_u32(st.vbase, st.voff + q);
        q += 4;
        if (l > (uint64_t)pg.val_len - q) { s_flag = 1; break; }
        if (k >= td.k0) s_vals[k - td.k0] = q | ((uint64_t)l << 32);
        q += l;
      }
    }
    __syncthreads();
    if (s_flag) { if (threadIdx.x == 0) set_err(err, ERR_STRING, td.page); return; }
  } else {
    const uint32_t rg = pg.chunk % (uint32_t)cs.nrg;
    const DictSlot sl = slots[cs.dict_slot0 + (rg - (uint32_t)cs.rg_begin)];
    if (sl.page == ~0u) { if (threadIdx.x == 0) set_err(err, ERR_DICT_MISSING, td.page); return; }
    src = sl.body;
    src_off = 0;
    if (td.nn > 0) {
      const uint32_t w = ld_u32(st.vbase, st.voff) & 0xff;
      const uint32_t* pairs = reinterpret_cast<const uint32_t*>(ws + sl.ws_entries);
      const uint32_t dn = sl.n;
      auto emit = [&](uint32_t i, uint32_t v, bool active, uint32_t) {
        if (!active) return;
        if (v >= dn) { s_flag = 1; v = 0; }
        s_vals[i] = (uint64_t)pairs[2 * v] | ((uint64_t)pairs[2 * v + 1] << 32);
      };
      if (!wg_hybrid(st.vbase, st.voff + td.val_pos, st.vend, td.val_skip, w, td.nn, false, s_runs, s_meta, &s_pos, err,
                     td.page, emit))
        return;
      __syncthreads();
      if (s_flag) { if (threadIdx.x == 0) set_err(err, ERR_DICT_INDEX, td.page); return; }
    }
  }

  // ---- offsets: exclusive scan of row lengths, thread j owns rows [16j, 16j+16) ----
  const uint64_t* aux = reinterpret_cast<const uint64_t*>(ws + cs.ws_tile_aux);
  const uint64_t base = aux[t - cs.tile_begin];
  constexpr int PER = TILE_ROWS / WG;
  uint64_t acc = 0;
  for (int q = 0; q < PER; ++q) {
    const uint32_t r = threadIdx.x * PER + q;
    if (r < nrows && (!opt || row_valid(s_valid, r))) acc += s_vals[opt ? row_rank(s_valid, s_pre, r) : r] >> 32;
  }
  uint64_t tot;
  uint64_t run = base + wg_excl_scan_u64(acc, s_tmp, &tot);
  const bool fits = base + tot <= cs.chars_capacity;
  for (int q = 0; q < PER; ++q) {
    const uint32_t r = threadIdx.x * PER + q;
    if (r >= nrows) break;
    if (cs.offsets) cs.offsets[out0 + r] = (int64_t)run;
    if (!opt || row_valid(s_valid, r)) {
      const uint64_t pv = s_vals[opt ? row_rank(s_valid, s_pre, r) : r];
      const uint32_t len = (uint32_t)(pv >> 32);
      const uint8_t* sp = src + src_off + (uint32_t)pv;
      if (fits && cs.chars) {
        uint8_t* dp = cs.chars + run;
        for (uint32_t b = 0; b < len; ++b) dp[b] = sp[b];
      }
      run += len;
    }
  }
}

}  // namespace pqk
