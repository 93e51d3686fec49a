// pq_open_kernels.hip -- kernels that run once when a file is opened:
//   k_walk   page-header walk of every column chunk -> device page table
//   k_index  tile index: entry positions of every TILE_ROWS-row tile in the
//            level and value streams of each data page, string checkpoints.
//   k_schain_cand / k_schain_link / k_schain_fill / k_schain_seq
//            string checkpoints of long dictionary pages, segments side by side
//   k_lv_cand / k_lv_link / k_lv_tiles
//            tile entries, level checkpoints and non-null counts of pages
//            with long definition-level streams, segments side by side
//   k_dl_cand / k_dl_link / k_dl_fill / k_dl_tiles
//            block positions, tile entries and block checkpoints of long
//            DELTA_BINARY_PACKED streams, segments side by side
//   k_di_cand / k_di_link / k_di_fill / k_di_ckpt
//            tile entries and value checkpoints of long dictionary-index
//            streams, segments side by side
#include <hip/hip_runtime.h>

#include "pq_device.hpp"
#include "pq_internal.h"

namespace pqk {

// Hybrid-run cursor used by the index pass (one lane).
struct RunCur {
  uint64_t hp;     // header position of the current run
  uint64_t next;   // position after the current run
  int64_t start;   // first value index of the current run
  uint64_t n;      // values in the run
  int bp;          // bit-packed?
  uint64_t pay;    // payload byte position (bit-packed)
  uint32_t val;    // RLE value
};

// Stream reader of one wave for k_index: all 64 lanes walk the same stream
// in lockstep (the walk is sequential; every lane computes the same values),
// served from a WIN-byte LDS window that the wave refills with coalesced
// 16-byte loads (one memory round trip per window instead of one per 16
// bytes); every read is an LDS read (all lanes read the same address, a
// broadcast).  The window keeps
// 256 bytes before the position that moved it, for the short look-backs of
// the walk (a run's payload).  Bytes at or past `lim` read as zero.
constexpr uint32_t WIN = 4096;
static_assert(NLCK == 64, "lane k of a wave writes level checkpoint k of a tile");
typedef uint32_t wr_u4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) wr_u4 lds_u4;

// Refills the window for position a (a multiple of 16); returns its start.
__device__ __noinline__ uint64_t wr_refill(const uint8_t* base, uint64_t lim, lds_u4* win, uint64_t a) {
  uint64_t wpos = a > 256 ? a - 256 : 0;
  wpos = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(wpos >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)wpos);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (uint32_t j = 0; j < WIN / 16 / 64; ++j) {
    const uint32_t k = lane + 64 * j;
    const uint64_t g = wpos + 16ull * k;
    wr_u4 v = {0u, 0u, 0u, 0u};
    if (g + 16 <= lim) v = *reinterpret_cast<const wr_u4*>(base + g);
    win[k] = v;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return wpos;
}

struct WR {
  const uint8_t* base;
  uint64_t lim;   // bytes of base that may be read (a multiple of 16)
  uint64_t wpos;  // window start (a multiple of 16)
  lds_u4* win;
  __device__ __forceinline__ void init(const uint8_t* b, uint64_t l, lds_u4* w) {
    base = b;
    lim = l;
    win = w;
    wpos = ~0ull;
  }
  // the window holds bytes [off, off + n)
  __device__ __forceinline__ void ensure(uint64_t off, uint32_t n) {
    if (off < wpos || off + n - wpos > WIN) wpos = wr_refill(base, lim, win, off & ~15ull);
  }
  // every lane reads the same byte, so the value is moved to a scalar
  // register: the walk that follows runs on the scalar unit, with scalar
  // branches instead of exec-mask updates
  __device__ __forceinline__ uint32_t byte(uint64_t off) {
    ensure(off, 1);
    return (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)reinterpret_cast<__attribute__((address_space(3))) uint8_t*>(win)[off - wpos]);
  }
  __device__ __forceinline__ uint32_t u32(uint64_t off) {
    ensure(off, 8);  // both aligned dwords holding bytes [off, off + 4)
    const uint32_t o = (uint32_t)(off - wpos);
    const __attribute__((address_space(3))) uint32_t* w32 = reinterpret_cast<__attribute__((address_space(3))) uint32_t*>(win);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)__builtin_amdgcn_alignbyte(w32[(o >> 2) + 1], w32[o >> 2], o & 3));
  }
};

// Wave reader with the window in registers: 256 bytes, four per lane; a
// read at a wave-uniform offset is one v_readlane, so a walk whose every
// position is wave-uniform waits on memory once per window, not per byte.
// Every lane must take part in every read.  It reads a global buffer
// readable up to lim (a multiple of 16); bytes at or past lim read as zero.
struct GRegWin {
  const uint8_t* base;
  uint64_t lim, wl;  // window start (a multiple of 4)
  uint32_t v;
  __device__ __forceinline__ void init(const uint8_t* b, uint64_t l) {
    base = b;
    lim = l;
    wl = 1ull << 63;  // far from every offset: the first read fills the window
    v = 0;
  }
  __device__ __forceinline__ uint32_t byte(uint64_t off) {
    if (off - wl >= 256) {
      wl = off & ~3ull;
      const uint64_t a = wl + 4ull * (threadIdx.x & 63);
      v = a + 4 <= lim ? *reinterpret_cast<const uint32_t*>(base + a) : 0u;
    }
    const uint32_t o = (uint32_t)(off - wl);
    return ((uint32_t)__builtin_amdgcn_readlane((int)v, (int)(o >> 2)) >> (8 * (o & 3))) & 0xffu;
  }
};

// The page table entry of a page whose header h was parsed, payload first.
__device__ __forceinline__ PageDev make_page(const PageHdr& h, uint64_t payload, uint32_t chunk) {
  PageDev p;
  p.payload = payload;
  p.comp_size = (uint32_t)h.comp;
  p.uncomp_size = (uint32_t)h.unc;
  p.num_values = h.nv;
  p.num_nulls = h.type == PAGE_DATA_V2 ? h.nnulls : -1;
  p.chunk = chunk;
  p.kind = (uint8_t)h.type;
  p.encoding = (uint8_t)h.enc;
  p.v2_compressed = (uint8_t)(h.type == PAGE_DATA_V2 ? h.is_comp : 1);
  p.flags = 0;
  p.def_len = h.type == PAGE_DATA_V2 ? h.def_len : 0;
  p.rep_len = h.type == PAGE_DATA_V2 ? h.rep_len : 0;
  p.def_off = 0; p.val_off = 0; p.val_len = 0;
  p.scratch_len = 0; p.scratch_off = 0; p.row0 = 0;
  p.tile_begin = 0; p.nonnull = 0; p.strck_begin = 0; p.dict_page = ~0u; p.dict_maxlen = 0;
  p.enc_w = 0; p.enc_m = 0; p.delta_first = 0; p.blocks_at = 0; p.sblk_begin = 0; p.chars_at = 0;
  p.x_src = 0; p.x_len = 0; p.x_sfx = 0; p.x_chars = 0; p.xlen = 0; p.x_total = 0; p.x_scratch = 0; p.x_off = 0;
  return p;
}

// One wave per column chunk.  Walks PageHeader, payload, PageHeader, ...
// from the chunk start until the chunk's byte range is consumed, checking
// every header.  With `pages == nullptr` it counts pages (first pass) and,
// when `rec` is given, records the header offsets of the first rec_cap[chunk]
// pages at rec[rec_base[chunk] ..] (setting *overflow past that); otherwise
// it writes the page table entries at page_base[chunk].  Each header is
// read through a register window that the wave fills with one coalesced
// load (the headers of a chunk lie a page apart, so a byte-serial reader
// would wait on memory for every 16 bytes); every lane parses, lane 0
// stores.
__global__ __launch_bounds__(64) void k_walk(const uint8_t* file, uint64_t file_lim, const ChunkDev* chunks,
                                             int nchunks, uint32_t* counts, const uint32_t* page_base,
                                             PageDev* pages, uint32_t* err, uint64_t* rec, const uint32_t* rec_base,
                                             const uint32_t* rec_cap, uint32_t* overflow) {
  const int q = blockIdx.x;
  if (q >= nchunks) return;
  const bool lead = threadIdx.x == 0;
  ChunkDev c = chunks[q];
  GRegWin r;
  r.init(file, file_lim);
  uint64_t pos = c.start;
  uint32_t n = 0;
  int64_t rows = 0;
  bool seen_data = false, seen_dict = false;
  const uint32_t cap = rec ? rec_cap[q] : 0u;
  while (pos < c.end) {
    PageHdr h;
    const uint64_t hpos = pos;
    if (!parse_page_header(r, pos, c.end, h) || h.type < 0 || h.unc < 0 || h.comp < 0) { if (lead) set_err(err, ERR_HEADER, q); return; }
    uint64_t payload = pos;
    if ((uint64_t)h.comp > c.end - payload) { if (lead) set_err(err, ERR_CHUNK_BOUNDS, q); return; }
    pos = payload + (uint64_t)h.comp;
    if (h.type == PAGE_DICT) {
      if (seen_data || seen_dict) { if (lead) set_err(err, ERR_PAGE_ORDER, q); return; }
      if (!h.has_sub || h.nv < 0) { if (lead) set_err(err, ERR_HEADER, q); return; }
      if (h.enc != E_PLAIN && h.enc != E_PLAIN_DICT) { if (lead) set_err(err, ERR_UNSUPPORTED, q); return; }
      if (c.codec == 0 && h.comp != h.unc) { if (lead) set_err(err, ERR_HEADER, q); return; }
      seen_dict = true;
    } else if (h.type == PAGE_DATA || h.type == PAGE_DATA_V2) {
      if (!h.has_sub || h.nv < 0) { if (lead) set_err(err, ERR_HEADER, q); return; }
      bool enc_ok = h.enc == E_PLAIN || h.enc == E_PLAIN_DICT || h.enc == E_RLE_DICT ||
                    (h.enc == E_DELTA && (c.type == T_INT32 || c.type == T_INT64)) ||
                    (h.enc == E_BSS && c.type != T_BYTE_ARRAY) ||
                    ((h.enc == E_DLBA || h.enc == E_DBA) && c.type == T_BYTE_ARRAY);
      // (DELTA_BYTE_ARRAY pages open, and are reported as unsupported only
      // when a scan selects their column)
      if (!enc_ok) { if (lead) set_err(err, ERR_UNSUPPORTED, q); return; }
      if (h.type == PAGE_DATA_V2) {
        if (h.rep_len != 0) { if (lead) set_err(err, ERR_UNSUPPORTED, q); return; }
        if (h.def_len < 0 || h.nrows != h.nv || h.def_len > h.comp || h.def_len > h.unc || h.nnulls < 0 ||
            (!c.optional && (h.def_len != 0 || h.nnulls != 0))) { if (lead) set_err(err, ERR_V2, q); return; }
        bool compressed = c.codec == 1 && h.is_comp;
        if (!compressed && h.comp != h.unc) { if (lead) set_err(err, ERR_V2, q); return; }
      } else if (c.codec == 0 && h.comp != h.unc) { if (lead) set_err(err, ERR_HEADER, q); return; }
      rows += h.nv;
      if (rows > c.rows) { if (lead) set_err(err, ERR_ROWS, q); return; }
      seen_data = true;
    } else {
      continue;  // index pages and unknown page types are skipped
    }
    if (pages) {
      const PageDev p = make_page(h, payload, (uint32_t)q);
      if (lead) pages[page_base[q] + n] = p;
    } else if (rec && lead) {
      if (n < cap) rec[rec_base[q] + n] = hpos;
      else *overflow = 1;
    }
    ++n;
  }
  if (pos != c.end || rows != c.rows) { if (lead) set_err(err, ERR_ROWS, q); return; }
  if (counts && lead) counts[q] = n;
}

// One lane per page recorded by k_walk's first pass: parses its header again
// (already checked there) into the page table.  page_chunk[i] is page i's
// chunk; its header offset is rec[rec_base[chunk] + i - page_base[chunk]].
__global__ void k_walk_rec(const uint8_t* file, const ChunkDev* chunks, const uint64_t* rec, const uint32_t* rec_base,
                           const uint32_t* page_base, const uint32_t* page_chunk, uint32_t npages, PageDev* pages,
                           uint32_t* err) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npages) return;
  const uint32_t q = page_chunk[i];
  const uint64_t end = chunks[q].end;
  uint64_t pos = rec[rec_base[q] + (i - page_base[q])];
  BR r;
  r.init(file);
  PageHdr h;
  if (!parse_page_header(r, pos, end, h)) { set_err(err, ERR_HEADER, q); return; }
  pages[i] = make_page(h, pos, q);
}

// Reads the run header at cur.next; returns false when the stream ends or a
// run leaves it.
__device__ inline bool run_next(WR& r, uint64_t end, uint32_t w, RunCur& c) {
  uint64_t pos = c.next;
  c.start += (int64_t)c.n;
  c.hp = pos;
  bool bad = false;
  uint64_t h = br_uleb(r, pos, end, bad);
  if (bad) return false;
  if (h & 1) {
    uint64_t g = h >> 1;
    if (g > (1ull << 28)) return false;
    c.bp = 1;
    c.n = g * 8;
    c.pay = pos;
    uint64_t nb = g * w;
    if (nb > end - pos) return false;
    c.next = pos + nb;
    c.val = 0;
  } else {
    c.bp = 0;
    c.n = h >> 1;
    uint32_t vb = (w + 7) / 8;
    if (vb > end - pos) return false;
    uint32_t v = 0;
    for (uint32_t j = 0; j < vb; ++j) v |= r.byte(pos + j) << (8 * j);
    c.val = v;
    c.pay = pos;
    c.next = pos + vb;
  }
  return true;
}

// number of set bits among the first `k` values of a bit-packed w=1 run
// (1024 bits per window check, then a dword per 32 bits straight from LDS)
__device__ inline uint32_t bp_popcount(WR& r, uint64_t pay, uint64_t k) {
  uint32_t s = 0;
  const __attribute__((address_space(3))) uint32_t* w32 =
      reinterpret_cast<const __attribute__((address_space(3))) uint32_t*>(r.win);
  for (uint64_t b0 = 0; b0 < k; b0 += 1024) {
    const uint32_t kk = (uint32_t)min(k - b0, (uint64_t)1024);
    const uint64_t off = pay + (b0 >> 3);
    r.ensure(off, 136);  // the 128 bytes and the dword after them
    const uint32_t o = (uint32_t)(off - r.wpos), sh = o & 3, d = o >> 2;
    for (uint32_t i = 0; 32 * i < kk; ++i) {
      uint32_t v = __builtin_amdgcn_alignbyte(w32[d + i + 1], w32[d + i], sh);
      const uint32_t left = kk - 32 * i;
      if (left < 32) v &= (1u << left) - 1u;
      s += __popc(v);
    }
  }
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)s);
}

// Checkpoint of value `target` inside run c of a w-bit hybrid stream whose
// tile entry sits at absolute position `entry`.
__device__ __forceinline__ Ck make_ck(const RunCur& c, int64_t target, uint32_t w, uint64_t entry, bool levels) {
  Ck k;
  k.at = CK_NONE;
  k.info = 0;
  const uint64_t skip = (uint64_t)(target - c.start);
  const uint64_t left = min(c.n - skip, (uint64_t)CK_LEFT);
  if (c.bp) {
    const uint64_t bit = c.pay * 8 + skip * w;
    const uint64_t off = (bit >> 3) - entry;
    if (off >= CK_NONE) return k;
    k.at = (uint32_t)off;
    k.info = 0x80000000u | ((uint32_t)(bit & 7) << 28) | (uint32_t)left;
  } else {
    const uint64_t off = c.hp - entry;
    if (off >= CK_NONE) return k;
    k.at = (uint32_t)off;
    k.info = (uint32_t)left | (levels ? ((1u << 29) | ((c.val & 1u) << 30)) : 0u);
  }
  return k;
}

// Level checkpoint (format in pq_internal.h) of row `target` inside run c of
// a level stream whose tile entry sits at absolute position `entry`.
__device__ __forceinline__ uint32_t make_lck(const RunCur& c, int64_t target, uint64_t entry) {
  const uint64_t skip = (uint64_t)(target - c.start);
  const uint64_t left = min(c.n - skip, (uint64_t)LROWS);
  uint64_t off;
  uint32_t x;
  if (c.bp) {
    const uint64_t bit = c.pay * 8 + skip;
    off = (bit >> 3) - entry;
    x = (1u << 19) | ((uint32_t)(bit & 7) << 16);
  } else {
    off = c.next - entry;
    x = (c.val & 1u) << 20;
  }
  if (off > 0xffffu) return LCK_NONE;
  return (uint32_t)off | x | ((uint32_t)left << 21);
}

__device__ __forceinline__ Ck ck_at(uint64_t off) {
  Ck k;
  k.at = off < CK_NONE ? (uint32_t)off : CK_NONE;
  k.info = 0;
  return k;
}

__device__ __forceinline__ Ck ck_none() {
  Ck k;
  k.at = CK_NONE;
  k.info = 0;
  return k;
}

// One wave per page (a 64-thread workgroup; every lane runs the same walk
// and stores the same values).  `scratch` holds every compressed page
// decompressed at its file-wide scratch offset; file_lim and scratch_lim are
// the readable bytes of the two buffers (multiples of 16).
__global__ __launch_bounds__(64) void k_index(const uint8_t* file, const uint8_t* scratch, PageDev* pages, int npages,
                                              const ChunkDev* chunks, TileDev* tiles, uint32_t* strck, uint32_t* ckl,
                                              Ck* ckv, uint32_t* err, uint64_t file_lim, uint64_t scratch_lim,
                                              const uint32_t* order, const uint8_t* xscratch, uint64_t xscratch_lim,
                                              int phase) {
  __shared__ wr_u4 s_win[WIN / 16];
  // DELTA pages of at most TC tiles: first value, value count and value
  // entry of every tile, so that the block walk reads no tile from memory
  constexpr uint32_t TC = 2048;
  __shared__ uint32_t s_k0[TC], s_nn[TC], s_vp[TC];
  if ((int)blockIdx.x >= npages) return;
  const int p = (int)order[blockIdx.x];  // workgroup i walks page order[i]
  PageDev pg = pages[p];
  ChunkDev ch = chunks[pg.chunk];
  const bool in_scratch = pg.scratch_len > 0;
  WR r;
  lds_u4* win = (lds_u4*)&s_win[0];
  // Stores that nothing in this kernel reads back (checkpoints) come from
  // lane 0 alone.
  // Tiles and the page entry are stored by every lane (each lane reads back
  // its own stores).
  const bool lead = (threadIdx.x & 63) == 0;
  auto lim_of = [&](const uint8_t* b) { return b == file ? file_lim : (b == xscratch ? xscratch_lim : scratch_lim); };

  if (pg.kind == PAGE_DICT) {
    const uint8_t* base = in_scratch ? scratch : file;
    uint64_t off = in_scratch ? pg.scratch_off : pg.payload;
    uint64_t blen = pg.uncomp_size;
    pg.val_off = off;
    pg.val_len = (uint32_t)blen;
    pg.flags = in_scratch ? 2 : 0;
    if (ch.type == T_BYTE_ARRAY && blen > SCHAIN_MIN) {
      pg.dict_maxlen = 0;  // the chain is walked by the k_schain kernels
    } else if (ch.type == T_BYTE_ARRAY) {
      // the length-prefix chain in 32-bit positions (a page is below 4 GiB):
      // q in the page body, o in the LDS window, one LDS read per entry; the
      // window moves when an entry's length prefix would leave it.  Every
      // lane reads the same length, which is moved to a scalar register, so
      // the chain and its checks run on the scalar unit
      const uint64_t blim = lim_of(base);
      const uint32_t n = pg.num_values > 0 ? (uint32_t)pg.num_values : 0u;
      const uint32_t bl = (uint32_t)blen;
      const __attribute__((address_space(3))) uint32_t* w32 =
          reinterpret_cast<const __attribute__((address_space(3))) uint32_t*>(win);
      uint32_t q = 0, maxlen = 0, k = 0;
      while (k < n) {
        const uint64_t wpos = wr_refill(base, blim, win, (off + q) & ~15ull);
        uint32_t o = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(off + q - wpos));  // below 272
        while (k < n && o + 8 <= WIN) {
          if ((k % STR_CK) == 0 && lead) strck[pg.strck_begin + k / STR_CK] = q;
          if (bl - q < 4) { set_err(err, ERR_STRING, p); return; }
          const uint32_t l = (uint32_t)__builtin_amdgcn_readfirstlane(
              (int)__builtin_amdgcn_alignbyte(w32[(o >> 2) + 1], w32[o >> 2], o & 3));
          if (l > bl - q - 4) { set_err(err, ERR_STRING, p); return; }
          q += 4 + l;
          o = l < WIN ? o + 4 + l : WIN;
          maxlen = max(maxlen, l);
          ++k;
        }
      }
      pg.dict_maxlen = maxlen;
    } else {
      uint64_t w = ch.type == T_INT32 ? 4 : 8;
      if ((uint64_t)pg.num_values * w > blen) { set_err(err, ERR_VALUES, p); return; }
    }
    pages[p] = pg;
    return;
  }

  // ---- stream layout of a data page ----
  // Pages with long level streams (lv_page) are indexed in two launches:
  // phase 1 stores their stream layout and leaves the levels to the k_lv
  // kernels, which store the tile entries, level checkpoints and non-null
  // count; phase 2 then indexes their value streams.
  const uint8_t* dbase = file;
  const uint8_t* vbase = file;
  uint64_t def_off = 0, def_len = 0, val_off = 0, val_len = 0;
  const bool lvp = lv_page(pg, ch.optional);
  if (phase == 2) {
    if (*(volatile uint32_t*)err != 0) return;  // the open has failed already
    vbase = (pg.flags & 4) ? xscratch : ((pg.flags & 2) ? scratch : file);
    def_off = pg.def_off;
    def_len = (uint64_t)pg.def_len;
    val_off = pg.val_off;
    val_len = pg.val_len;
  } else {
    if (pg.kind == PAGE_DATA) {
      const uint8_t* base = in_scratch ? scratch : file;
      uint64_t off = in_scratch ? pg.scratch_off : pg.payload;
      uint64_t blen = pg.uncomp_size;
      dbase = vbase = base;
      r.init(base, lim_of(base), win);
      if (ch.optional) {
        if (blen < 4) { set_err(err, ERR_LEVELS, p); return; }
        uint64_t L = r.u32(off);
        if (L > blen - 4) { set_err(err, ERR_LEVELS, p); return; }
        def_off = off + 4; def_len = L;
        val_off = off + 4 + L; val_len = blen - 4 - L;
      } else {
        val_off = off; val_len = blen;
      }
      pg.flags = in_scratch ? 3 : 0;
    } else {
      dbase = file;
      def_off = pg.payload + (uint64_t)pg.rep_len;
      def_len = (uint64_t)pg.def_len;
      if (in_scratch) {
        vbase = scratch;
        val_off = pg.scratch_off;
        val_len = pg.scratch_len;
        pg.flags = 2;
      } else {
        vbase = file;
        val_off = def_off + def_len;
        val_len = pg.comp_size - (uint64_t)pg.rep_len - def_len;
        pg.flags = 0;
      }
    }
    if (pg.encoding == E_DBA && ch.type == T_BYTE_ARRAY && pg.x_total == DBA_UNSUPPORTED) {
      pg.encoding = E_UNDECODED;  // reported by the decode kernels when the column is scanned
    } else if (pg.encoding == E_DBA && ch.type == T_BYTE_ARRAY) {
      // DELTA_BYTE_ARRAY: the values, expanded to the PLAIN layout by k_dba,
      // are indexed and decoded like a PLAIN page
      vbase = xscratch;
      val_off = pg.x_off;
      val_len = pg.xlen;
      pg.flags = (uint8_t)((pg.flags & 1) | 4);
    }
    pg.def_off = def_off;
    pg.def_len = (int32_t)def_len;
    pg.val_off = val_off;
    pg.val_len = (uint32_t)val_len;
    if (lvp) {
      pages[p] = pg;
      return;
    }
  }

  const int64_t nv = pg.num_values;
  const uint32_t ntiles = (uint32_t)((nv + TILE_ROWS - 1) / TILE_ROWS);

  // ---- definition levels: tile entry points, sub-tile checkpoints, non-null counts ----
  uint32_t nonnull = 0;
  if (phase == 2) {
    nonnull = pg.nonnull;
  } else if (ch.optional) {
    r.init(dbase, lim_of(dbase), win);
    const uint64_t end = def_off + def_len;
    RunCur c;
    c.next = def_off; c.start = 0; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0; c.hp = def_off;
    uint64_t before = 0;  // valid rows in runs before the current one
    bool have = false;
    TileDev td;
    for (int64_t target = 0; target < nv; target += LROWS) {
      while (!have || c.start + (int64_t)c.n <= target) {
        if (have) before += c.bp ? bp_popcount(r, c.pay, c.n) : (uint64_t)c.val * c.n;
        if (!run_next(r, end, 1, c) || (!c.bp && c.val > 1)) { set_err(err, ERR_LEVELS, p); return; }
        have = true;
      }
      const uint64_t skip = (uint64_t)(target - c.start);
      const uint32_t t = (uint32_t)(target / TILE_ROWS), sub = (uint32_t)((target % TILE_ROWS) / LROWS);
      if (sub == 0) {
        td.page = (uint32_t)p;
        td.row0 = (uint32_t)target;
        td.k0 = (uint32_t)(before + (c.bp ? bp_popcount(r, c.pay, skip) : (uint64_t)c.val * skip));
        td.nn = 0;
        td.def_pos = (uint32_t)(c.hp - def_off);
        td.def_skip = (uint32_t)skip;
        td.val_pos = 0;
        td.val_skip = 0;
        tiles[pg.tile_begin + t] = td;
      }
      if (lead) ckl[(size_t)(pg.tile_begin + t) * NLCK + sub] = make_lck(c, target, def_off + td.def_pos);
    }
    // the last tile's checkpoints past the page's rows
    if (nv > 0 && lead)
      for (int64_t target = ((nv + LROWS - 1) / LROWS) * LROWS; target % TILE_ROWS != 0; target += LROWS)
        ckl[(size_t)(pg.tile_begin + (uint32_t)(target / TILE_ROWS)) * NLCK + (target % TILE_ROWS) / LROWS] = LCK_NONE;
    if (nv > 0) {
      while (!have || c.start + (int64_t)c.n < nv) {
        if (have) before += c.bp ? bp_popcount(r, c.pay, c.n) : (uint64_t)c.val * c.n;
        if (!run_next(r, end, 1, c) || (!c.bp && c.val > 1)) { set_err(err, ERR_LEVELS, p); return; }
        have = true;
      }
      const uint64_t part = (uint64_t)(nv - c.start);
      nonnull = (uint32_t)(before + (c.bp ? bp_popcount(r, c.pay, part) : (uint64_t)c.val * part));
    }
  } else {
    nonnull = (uint32_t)nv;
    for (uint32_t t = 0; t < ntiles; ++t) {
      TileDev td;
      td.page = (uint32_t)p;
      td.row0 = t * TILE_ROWS;
      td.k0 = t * TILE_ROWS;
      td.nn = 0;
      td.def_pos = 0; td.def_skip = 0; td.val_pos = 0; td.val_skip = 0;
      tiles[pg.tile_begin + t] = td;
      ckl[(size_t)(pg.tile_begin + t) * NLCK + (threadIdx.x & 63)] = LCK_NONE;  // lane k: checkpoint k
    }
  }
  if (lead)
    for (uint32_t t = 0; t < ntiles; ++t)
      for (int k = 0; k < NSUB; ++k) ckv[(size_t)(pg.tile_begin + t) * NSUB + k] = ck_none();
  if (pg.kind == PAGE_DATA_V2 && (int64_t)pg.num_nulls != nv - (int64_t)nonnull) { set_err(err, ERR_V2, p); return; }
  pg.nonnull = nonnull;
  for (uint32_t t = 0; t < ntiles; ++t) {
    uint32_t k0 = tiles[pg.tile_begin + t].k0;
    uint32_t k1 = t + 1 < ntiles ? tiles[pg.tile_begin + t + 1].k0 : nonnull;
    tiles[pg.tile_begin + t].nn = k1 - k0;
  }

  // ---- value stream entry points ----
  r.init(vbase, lim_of(vbase), win);
  const uint64_t vend = val_off + val_len;
  const int enc = pg.encoding;
  if ((enc == E_PLAIN || enc == E_BSS) && ch.type != T_BYTE_ARRAY) {
    uint64_t w = ch.type == T_INT32 ? 4 : 8;
    if ((uint64_t)nonnull * w > val_len) { set_err(err, ERR_VALUES, p); return; }
  } else if (enc == E_PLAIN || enc == E_DBA) {
    if (enc == E_DBA && pg.x_total != nonnull) { set_err(err, ERR_VALUES, p); return; }
    uint64_t q = val_off;
    uint32_t t = 0;
    for (uint32_t k = 0; k <= nonnull; ++k) {
      while (t < ntiles && tiles[pg.tile_begin + t].k0 == k) {
        tiles[pg.tile_begin + t].val_pos = (uint32_t)(q - val_off);
        if (t > 0) tiles[pg.tile_begin + t - 1].val_skip = (uint32_t)(q - val_off);
        ++t;
      }
      if (k == nonnull) break;
      if ((k % STR_CK) == 0 && lead) strck[pg.strck_begin + k / STR_CK] = (uint32_t)(q - val_off);
      if (vend - q < 4) { set_err(err, ERR_STRING, p); return; }
      uint32_t l = r.u32(q);
      q += 4;
      if (l > vend - q) { set_err(err, ERR_STRING, p); return; }
      q += l;
    }
    if (ntiles > 0) tiles[pg.tile_begin + ntiles - 1].val_skip = (uint32_t)(q - val_off);
  } else if (enc == E_PLAIN_DICT || enc == E_RLE_DICT) {
    if (pg.dict_page == ~0u) { set_err(err, ERR_DICT_MISSING, p); return; }
    if (nonnull > 0) {
      if (val_len < 1) { set_err(err, ERR_VALUES, p); return; }
      const uint32_t w = r.byte(val_off);
      if (w > 32) { set_err(err, ERR_VALUES, p); return; }
      pg.enc_w = w;
      if (di_page(pg)) {  // long index stream: walked by the k_di kernels
        pages[p] = pg;
        return;
      }
      RunCur c;
      c.next = val_off + 1; c.start = 0; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0; c.hp = val_off + 1;
      bool have = false;
      for (uint32_t t = 0; t < ntiles; ++t) {
        TileDev& tdr = tiles[pg.tile_begin + t];
        const uint32_t k0 = tdr.k0, nnt = tdr.nn;
        for (uint32_t sub = 0; sub < NSUB && sub * SUB_ROWS < nnt; ++sub) {
          const int64_t target = (int64_t)k0 + (int64_t)sub * SUB_ROWS;
          while (!have || c.start + (int64_t)c.n <= target) {
            if (!run_next(r, vend, w, c)) { set_err(err, ERR_VALUES, p); return; }
            have = true;
          }
          if (sub == 0) {
            tdr.val_pos = (uint32_t)(c.hp - val_off);
            tdr.val_skip = (uint32_t)(target - c.start);
          }
          if (lead) ckv[(size_t)(pg.tile_begin + t) * NSUB + sub] = make_ck(c, target, w, val_off + tdr.val_pos, false);
        }
      }
      while (!have || c.start + (int64_t)c.n < (int64_t)nonnull) {
        if (!run_next(r, vend, w, c)) { set_err(err, ERR_VALUES, p); return; }
        have = true;
      }
    }
  } else if (enc == E_DELTA || (enc == E_DLBA && ch.type == T_BYTE_ARRAY)) {
    // DELTA_BINARY_PACKED values, or the lengths of DELTA_LENGTH_BYTE_ARRAY
    // strings (32-bit), whose chars follow the stream
    bool bad = false;
    uint64_t q = val_off;
    uint64_t B = br_uleb(r, q, vend, bad), M = br_uleb(r, q, vend, bad), total = br_uleb(r, q, vend, bad);
    const int64_t first = unzz(br_uleb(r, q, vend, bad));
    if (bad || B == 0 || B % 128 != 0 || M == 0 || B % M != 0 || (B / M) % 32 != 0 || total != nonnull) {
      set_err(err, ERR_DELTA, p);
      return;
    }
    if (M > 16 || B > 65536) { set_err(err, ERR_UNSUPPORTED, p); return; }
    const uint32_t maxw = ch.type == T_INT64 ? 64 : 32;
    const uint64_t per = B / M;
    pg.enc_w = (uint32_t)B;
    pg.enc_m = (uint32_t)M;
    pg.delta_first = first;
    pg.blocks_at = (uint32_t)(q - val_off);
    // block b holds values [1 + b*B, 1 + (b+1)*B); value 0 is in the header
    const uint64_t nblocks = total > 1 ? (total - 1 + B - 1) / B : 0;
    const bool cached = ntiles <= TC;
    for (uint32_t t = 0; t < ntiles; ++t) {
      tiles[pg.tile_begin + t].val_pos = (uint32_t)(q - val_off);
      tiles[pg.tile_begin + t].val_skip = 0;
      if (cached) {  // every lane wrote every tile above, so each reads its own stores
        s_k0[t] = tiles[pg.tile_begin + t].k0;
        s_nn[t] = tiles[pg.tile_begin + t].nn;
        s_vp[t] = (uint32_t)(q - val_off);
      }
    }
    if (dl_page(pg, ch.type)) {  // long chain: walked by the k_dl kernels
      pages[p] = pg;
      return;
    }
    auto tile_k0 = [&](uint32_t x) { return cached ? s_k0[x] : tiles[pg.tile_begin + x].k0; };
    auto tile_nn = [&](uint32_t x) { return cached ? s_nn[x] : tiles[pg.tile_begin + x].nn; };
    auto tile_vp = [&](uint32_t x) { return cached ? s_vp[x] : tiles[pg.tile_begin + x].val_pos; };
    uint32_t t = 0, ulo = 0;
    for (uint64_t b = 0; b < nblocks; ++b) {
      while (t < ntiles) {
        const uint32_t k0t = tile_k0(t), nnt = tile_nn(t);
        const uint64_t last = (uint64_t)k0t + nnt;  // one past the tile's last value
        if (nnt == 0 || last <= 1) { ++t; continue; }  // needs no block
        const uint64_t first = k0t == 0 ? 1 : k0t;
        const uint64_t nb = (first - 1) / B;
        if (nb != b) break;
        tiles[pg.tile_begin + t].val_pos = (uint32_t)(q - val_off);
        tiles[pg.tile_begin + t].val_skip = (uint32_t)((first - 1) % B);
        if (cached) s_vp[t] = (uint32_t)(q - val_off);
        ++t;
      }
      // this block's header, as checkpoint (b - entry block) of every tile
      // entered so far whose deltas reach block b; tiles before `ulo` end
      // before it
      while (ulo < t) {
        const uint32_t k0u = tile_k0(ulo), nnu = tile_nn(ulo);
        if (nnu != 0 && (uint64_t)k0u + nnu > 1 && ((uint64_t)k0u + nnu - 2) / B >= b) break;
        ++ulo;
      }
      for (uint32_t u = ulo; u < t; ++u) {
        TileDev tu;
        tu.k0 = tile_k0(u);
        tu.nn = tile_nn(u);
        tu.val_pos = tile_vp(u);
        if (tu.nn == 0 || (uint64_t)tu.k0 + tu.nn <= 1) continue;
        const uint64_t fu = tu.k0 == 0 ? 1 : tu.k0;
        const uint64_t bu = (fu - 1) / B;                    // entry block of tile u
        const uint64_t lastb = ((uint64_t)tu.k0 + tu.nn - 2) / B;  // block of its last delta
        if (b >= bu && b <= lastb && b - bu < NSUB && lead)
          ckv[(size_t)(pg.tile_begin + u) * NSUB + (b - bu)] = ck_at(q - val_off - tu.val_pos);
      }
      br_uleb(r, q, vend, bad);  // min delta
      if (bad || M > vend - q) { set_err(err, ERR_DELTA, p); return; }
      const uint64_t left = total - 1 - b * B;  // values from this block on
      const uint64_t used = left < B ? left : B;
      const uint64_t used_mb = (used + per - 1) / per;
      uint64_t body = 0;
      for (uint64_t m = 0; m < used_mb; ++m) {
        const uint32_t w = r.byte(q + m);
        if (w > maxw) { set_err(err, ERR_DELTA, p); return; }
        body += per * w / 8;
      }
      q += M;
      if (body > vend - q) { set_err(err, ERR_DELTA, p); return; }
      q += body;
    }
    pg.chars_at = (uint32_t)(q - val_off);
  }
  pages[p] = pg;
}


// ---------------------------------------------------------------------------
// Long string dictionary pages.  The body is a chain of (u32 length, bytes)
// entries whose positions are only known by walking it from the start.  The
// body is cut into SCHAIN_SEG-byte segments; in each segment, lane c walks
// the chain that starts at byte c of the segment until it leaves the
// segment (k_schain_cand).  The true chain enters a segment at most
// SCHAIN_CAND - 1 bytes past its start unless an entry longer than that
// crosses the boundary, so one of the candidates is the true chain's walk;
// k_schain_link follows the true chain from segment to segment through the
// candidates' exits and gives each segment its entry position and entry
// index, and k_schain_fill walks each segment once more from there, storing
// a checkpoint every STR_CK entries.  A page whose true chain enters a
// segment past the candidates (or breaks) is walked whole by k_schain_seq.
// ---------------------------------------------------------------------------
constexpr uint32_t SCHAIN_LDS = SCHAIN_SEG + 64;

// Stages body bytes [s0, s0 + SCHAIN_SEG + 8) into LDS (16-byte chunks from
// the one holding byte s0; bytes at or past the readable limit read as
// zero); returns the LDS offset of byte s0.
__device__ __forceinline__ uint32_t schain_stage(const SChainPage& sp, uint32_t s0, uint8_t* lds) {
  const uint64_t g = sp.off + s0;
  const uint64_t a0 = g & ~15ull;
  for (uint32_t c = threadIdx.x; 16 * c < SCHAIN_SEG + 32; c += 64) {
    const uint64_t a = a0 + 16ull * c;
    wr_u4 v = {0u, 0u, 0u, 0u};
    if (a + 16 <= sp.lim) v = *reinterpret_cast<const wr_u4*>(sp.base + a);
    *(lds_u4*)(lds + 16 * c) = v;
  }
  __syncthreads();
  return (uint32_t)(g - a0);
}

__device__ __forceinline__ uint32_t schain_u32(const uint8_t* lds, uint32_t o) {
  const __attribute__((address_space(3))) uint32_t* w = (const __attribute__((address_space(3))) uint32_t*)lds;
  return __builtin_amdgcn_alignbyte(w[(o >> 2) + 1], w[o >> 2], o & 3);
}

__global__ __launch_bounds__(64) void k_schain_cand(const SChainPage* pgs, const uint32_t* seg_page, SChainCand* cand) {
  __shared__ __align__(16) uint8_t s_seg[SCHAIN_LDS];
  const uint32_t sg = blockIdx.x, c = threadIdx.x;
  const SChainPage sp = pgs[seg_page[sg]];
  const uint32_t s0 = (sg - sp.seg0) * SCHAIN_SEG;
  const uint32_t se = min(s0 + SCHAIN_SEG, sp.len);
  const uint8_t* lds = (const uint8_t*)&s_seg[0];
  const uint32_t lead = schain_stage(sp, s0, &s_seg[0]);
  uint32_t q = s0 + c, count = 0, maxlen = 0, state = q < se ? 0u : 1u;
  while (q < se) {
    if (sp.len - q < 4) { state = 1; break; }
    const uint32_t l = schain_u32(lds, lead + (q - s0));
    if (l > sp.len - q - 4) { state = 2; break; }
    q += 4 + l;
    ++count;
    maxlen = max(maxlen, l);
  }
  cand[(size_t)sg * SCHAIN_CAND + c] = SChainCand{q, count, maxlen, state};
}

// One thread per page.  ok[page] = 1 when every segment's entry was found
// among the candidates (then seg_start / seg_base hold each segment's first
// entry position and index, SCHAIN_NONE where no entry starts).
__global__ void k_schain_link(const SChainPage* pgs, int npg, const SChainCand* cand, uint32_t* seg_start,
                              uint32_t* seg_base, uint32_t* ok) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npg) return;
  const SChainPage sp = pgs[i];
  uint32_t q = 0, k = 0, good = 1;
  for (uint32_t j = 0; j < sp.nseg; ++j) {
    const uint32_t s0 = j * SCHAIN_SEG, se = min(s0 + SCHAIN_SEG, sp.len);
    seg_start[sp.seg0 + j] = SCHAIN_NONE;
    if (k >= sp.n || q >= se) continue;  // the chain has ended, or an entry covers the segment
    const uint32_t c = q - s0;
    if (c >= SCHAIN_CAND) { good = 0; break; }
    seg_start[sp.seg0 + j] = q;
    seg_base[sp.seg0 + j] = k;
    const SChainCand cd = cand[(size_t)(sp.seg0 + j) * SCHAIN_CAND + c];
    if (sp.n - k <= cd.count) { k = sp.n; continue; }  // the chain's last entry starts here
    if (cd.state != 0) { good = 0; break; }             // broken before its last entry
    q = cd.exit;
    k += cd.count;
  }
  if (k < sp.n) good = 0;  // ran out of body: the sequential walk reports it
  ok[i] = good;
}

// One workgroup per segment of a linked page: lane 0 walks the segment's
// entries from its first one, storing the checkpoints; the page's longest
// length is the maximum over its segments.
__global__ __launch_bounds__(64) void k_schain_fill(const SChainPage* pgs, const uint32_t* seg_page,
                                                    const uint32_t* seg_start, const uint32_t* seg_base,
                                                    const uint32_t* ok, uint32_t* strck, PageDev* pages, uint32_t* err) {
  __shared__ __align__(16) uint8_t s_seg[SCHAIN_LDS];
  const uint32_t sg = blockIdx.x;
  const uint32_t pi = seg_page[sg];
  if (!ok[pi] || seg_start[sg] == SCHAIN_NONE) return;
  const SChainPage sp = pgs[pi];
  const uint32_t s0 = (sg - sp.seg0) * SCHAIN_SEG;
  const uint32_t se = min(s0 + SCHAIN_SEG, sp.len);
  const uint8_t* lds = (const uint8_t*)&s_seg[0];
  const uint32_t lead = schain_stage(sp, s0, &s_seg[0]);
  if (threadIdx.x != 0) return;
  uint32_t q = seg_start[sg], k = seg_base[sg], maxlen = 0;
  while (q < se && k < sp.n) {
    if ((k % STR_CK) == 0) strck[sp.strck_begin + k / STR_CK] = q;
    if (sp.len - q < 4) { set_err(err, ERR_STRING, sp.page); return; }
    const uint32_t l = schain_u32(lds, lead + (q - s0));
    if (l > sp.len - q - 4) { set_err(err, ERR_STRING, sp.page); return; }
    q += 4 + l;
    maxlen = max(maxlen, l);
    ++k;
  }
  atomicMax(&pages[sp.page].dict_maxlen, maxlen);
}

// One wave per page that could not be linked: the whole chain, front to
// back, through an LDS window (as k_index walks the short pages).
__global__ __launch_bounds__(64) void k_schain_seq(const SChainPage* pgs, int npg, const uint32_t* ok, uint32_t* strck,
                                                   PageDev* pages, uint32_t* err) {
  __shared__ wr_u4 s_win[WIN / 16];
  const int i = blockIdx.x;
  if (i >= npg || ok[i]) return;
  const SChainPage sp = pgs[i];
  lds_u4* win = (lds_u4*)&s_win[0];
  const bool lead = (threadIdx.x & 63) == 0;
  const __attribute__((address_space(3))) uint32_t* w32 =
      reinterpret_cast<const __attribute__((address_space(3))) uint32_t*>(win);
  uint32_t q = 0, maxlen = 0, k = 0;
  const uint32_t n = sp.n, bl = sp.len;
  while (k < n) {
    const uint64_t wpos = wr_refill(sp.base, sp.lim, win, (sp.off + q) & ~15ull);
    uint32_t o = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(sp.off + q - wpos));
    while (k < n && o + 8 <= WIN) {
      if ((k % STR_CK) == 0 && lead) strck[sp.strck_begin + k / STR_CK] = q;
      if (bl - q < 4) { set_err(err, ERR_STRING, sp.page); return; }
      const uint32_t l = (uint32_t)__builtin_amdgcn_readfirstlane(
          (int)__builtin_amdgcn_alignbyte(w32[(o >> 2) + 1], w32[o >> 2], o & 3));
      if (l > bl - q - 4) { set_err(err, ERR_STRING, sp.page); return; }
      q += 4 + l;
      o = l < WIN ? o + 4 + l : WIN;
      maxlen = max(maxlen, l);
      ++k;
    }
  }
  if (lead) pages[sp.page].dict_maxlen = maxlen;
}

// ---------------------------------------------------------------------------
// Long definition-level streams.  The levels of an OPTIONAL page are a chain
// of hybrid runs of 1-bit values (a ULEB128 header; bit-packed: groups of 8
// values, one byte each; RLE: a count and one value byte), cut here into
// LV_SEG-byte segments.  k_lv_cand: lane c of a segment's workgroup walks the
// chain that starts at byte c of the segment, summing the rows and valid rows
// of the runs whose header lies in the segment, until it leaves it.  Runs are
// short (a bit-packed run of 63 groups takes 65 bytes), so the true chain
// enters each segment within its first LV_CAND bytes.  A chain that does not
// start at a run header soon reads an RLE value above 1 and stops, or meets
// a true header and goes on as the true chain: chains that reach the same
// header past the candidates' start bytes are walked from there once.
// k_lv_link follows the true chain from segment to segment through the
// candidates' exits, up to the run that covers the page's last row.
// k_lv_tiles (mode 0) then indexes a segment with one wave: lane 0 finds the
// first run header in each of its 64 sub-segments, each lane sums the valid
// rows of its sub-segment's runs, and each lane walks them once more,
// storing the entries of the tiles whose first row lies in them with the 64
// level checkpoints of each such tile and, at the page's last row, the
// non-null count.  A page whose chain leaves the candidates is walked whole
// by one wave (mode 1).
// ---------------------------------------------------------------------------
constexpr uint32_t LV_XTRA = 1024;  // bytes staged past a segment, for the runs that leave it
constexpr uint32_t LV_LDS = LV_SEG + LV_XTRA + 64;
constexpr uint32_t LV_SUB = LV_SEG / 64;  // sub-segment bytes (one lane each)
static_assert(LV_CAND <= LV_SEG && LV_CAND % 64 == 0, "candidates: whole waves inside a segment");

struct LvStream {
  const uint8_t* base;
  uint64_t lim;  // readable bytes of base (a multiple of 16)
  uint64_t off;  // stream offset in base
  uint32_t len;  // stream bytes
  int64_t nv;    // rows of the page
};
__device__ __forceinline__ LvStream lv_stream(const PageDev* pages, uint32_t p, const uint8_t* file,
                                              const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim) {
  LvStream st;
  const bool sc = (pages[p].flags & 1) != 0;  // V1 page body decompressed to scratch
  st.base = sc ? scratch : file;
  st.lim = sc ? scratch_lim : file_lim;
  st.off = pages[p].def_off;
  st.len = pages[p].def_len > 0 ? (uint32_t)pages[p].def_len : 0u;
  st.nv = pages[p].num_values;
  return st;
}
__device__ __forceinline__ uint32_t lv_sat(uint32_t a, uint64_t b) {
  const uint64_t x = (uint64_t)a + b;  // b < 2^63
  return x > 0xffffffffull ? 0xffffffffu : (uint32_t)x;
}

// Stages stream bytes [s0, sh) of st in LDS (16-byte chunks from the one
// holding byte s0; bytes at or past the readable limit read as zero), with
// `nthr` threads; returns d such that stream byte x sits at LDS byte d + x
// (32-bit wrap-around).
__device__ __forceinline__ uint32_t lv_stage(const LvStream& st, uint32_t s0, uint32_t sh, uint8_t* lds, uint32_t nthr) {
  const uint64_t g0 = st.off + s0, a0 = g0 & ~15ull, ga = st.off + sh;
  for (uint32_t k = threadIdx.x; a0 + 16ull * k < ga; k += nthr) {
    const uint64_t a = a0 + 16ull * k;
    wr_u4 v = {0u, 0u, 0u, 0u};
    if (a + 16 <= st.lim) v = *reinterpret_cast<const wr_u4*>(st.base + a);
    *(lds_u4*)(&lds[16 * k]) = v;
  }
  return (uint32_t)(g0 - a0) - s0;
}

// A run header of at most 4 bytes, decoded from the 4 bytes wv that start
// with it: returns its length (0: longer, read it byte by byte) and sets h.
__device__ __forceinline__ uint32_t uleb4(uint32_t wv, uint32_t& h) {
  const uint32_t cont = ~wv & 0x80808080u;  // bytes that end the header
  if (cont == 0) return 0;
  const uint32_t hl = (__builtin_ctz(cont) >> 3) + 1;
  const uint32_t hv = (wv & 0x7fu) | ((wv >> 1) & 0x3f80u) | ((wv >> 2) & 0x1fc000u) | ((wv >> 3) & 0xfe00000u);
  h = hl == 4 ? hv : hv & ((1u << (7 * hl)) - 1u);
  return hl;
}

// One workgroup of LV_CAND lanes per segment; the segment and LV_XTRA bytes
// after it are staged in LDS.
__global__ __launch_bounds__(LV_CAND) void k_lv_cand(const LvPage* lps, const uint32_t* seg_page, const PageDev* pages,
                                                     const uint8_t* file, const uint8_t* scratch, uint64_t file_lim,
                                                     uint64_t scratch_lim, LvCand* cand) {
  __shared__ __align__(16) uint8_t s_seg[LV_LDS];
  __shared__ uint32_t s_p1[LV_CAND], s_exit[LV_CAND], s_state[LV_CAND], s_rows[LV_CAND], s_valid[LV_CAND];
  const uint32_t sg = blockIdx.x, c = threadIdx.x;
  const LvPage lp = lps[seg_page[sg]];
  const LvStream st = lv_stream(pages, lp.page, file, scratch, file_lim, scratch_lim);
  const uint32_t s0 = (sg - lp.seg0) * LV_SEG;
  LvCand out = {s0 + c, 0u, 0u, 0u};
  if (s0 < st.len) {
    const uint32_t se = min(s0 + LV_SEG, st.len);           // run headers of this segment: [s0, se)
    const uint32_t sh = min(s0 + LV_SEG + LV_XTRA, st.len);  // staged stream bytes: [s0, sh)
    const bool to_end = sh == st.len;                        // the staged bytes reach the stream's end
    const uint32_t d = lv_stage(st, s0, sh, &s_seg[0], LV_CAND);
    __syncthreads();
    const __attribute__((address_space(3))) uint32_t* w32 = (const __attribute__((address_space(3))) uint32_t*)&s_seg[0];
    // walks the runs whose header lies before `lim` from q, adding their rows
    // and valid rows; 0 when it got there, 1 at an invalid run, 2 at a run
    // the staged bytes do not hold
    auto walk = [&](uint32_t& q, uint32_t lim, uint32_t& rows, uint32_t& valid) -> uint32_t {
      while (q < lim) {
        uint64_t h = 0;
        uint32_t x = q;
        bool whole = false;
        for (uint32_t b7 = 0; b7 < 70; b7 += 7) {
          if (x >= sh) return to_end ? 1u : 2u;
          const uint32_t b = s_seg[d + x];
          ++x;
          if (b7 == 63 && (b & 0x7e)) return 1;
          h |= (uint64_t)(b & 0x7f) << b7;
          if (!(b & 0x80)) { whole = true; break; }
        }
        if (!whole) return 1;
        if (h & 1) {
          const uint64_t g = h >> 1;  // payload bytes
          if (g > (1ull << 28) || g > st.len - x) return 1;
          if (x + g > sh) return 2;
          uint32_t cnt = 0;
          const uint32_t o = d + x;
          for (uint32_t i = 0; i < (uint32_t)g; i += 4) {
            uint32_t v = __builtin_amdgcn_alignbyte(w32[((o + i) >> 2) + 1], w32[(o + i) >> 2], (o + i) & 3);
            if ((uint32_t)g - i < 4) v &= (1u << (8 * ((uint32_t)g - i))) - 1u;
            cnt += __popc(v);
          }
          rows = lv_sat(rows, 8 * g);
          valid = lv_sat(valid, cnt);
          q = x + (uint32_t)g;
        } else {
          if (x >= st.len) return 1;
          if (x >= sh) return 2;
          const uint32_t v = s_seg[d + x];
          if (v > 1) return 1;
          rows = lv_sat(rows, h >> 1);
          if (v) valid = lv_sat(valid, h >> 1);
          q = x + 1;
        }
      }
      return 0;
    };
    uint32_t q = s0 + c, rows = 0, valid = 0;
    const uint32_t state = walk(q, min(se, s0 + LV_CAND), rows, valid);
    const uint32_t p1 = (state == 0 && q < se) ? q : LV_NONE;  // first header past the start bytes
    s_p1[c] = p1;
    __syncthreads();
    uint32_t lead = c;  // the first candidate that reached the same header
    if (p1 != LV_NONE)
      for (uint32_t k = 0; k < c; ++k)
        if (s_p1[k] == p1) { lead = k; break; }
    if (p1 != LV_NONE && lead == c) {
      uint32_t q2 = q, r2 = 0, v2 = 0;
      s_state[c] = walk(q2, se, r2, v2);
      s_exit[c] = q2;
      s_rows[c] = r2;
      s_valid[c] = v2;
    }
    __syncthreads();
    out = p1 != LV_NONE ? LvCand{s_exit[lead], s_state[lead], lv_sat(rows, s_rows[lead]), lv_sat(valid, s_valid[lead])}
                        : LvCand{q, state, rows, valid};
  }
  cand[(size_t)sg * LV_CAND + c] = out;
}

// One thread per page: the true chain's entry into each segment it crosses,
// up to the run covering the page's last row.  ok[page] = 0 when the chain
// enters a segment past its candidates or meets a run the candidates could
// not follow; then no segment is walked and k_lv_tiles walks the page whole.
__global__ void k_lv_link(const LvPage* lps, int npg, const PageDev* pages, const LvCand* cand, LvEntry* ent,
                          uint32_t* ok, uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npg) return;
  const LvPage lp = lps[i];
  const uint32_t len = pages[lp.page].def_len > 0 ? (uint32_t)pages[lp.page].def_len : 0u;
  const uint64_t nv = (uint64_t)pages[lp.page].num_values;
  for (uint32_t j = 0; j < lp.nseg; ++j) ent[lp.seg0 + j].q = LV_NONE;
  uint32_t q = 0, good = 1;
  uint64_t R = 0, V = 0;
  for (;;) {
    if (q >= len) { set_err(err, ERR_LEVELS, lp.page); break; }  // the levels end before the last row
    const uint32_t j = q / LV_SEG, c = q % LV_SEG;
    if (j >= lp.nseg || c >= LV_CAND) { good = 0; break; }
    const LvCand cd = cand[(size_t)(lp.seg0 + j) * LV_CAND + c];
    ent[lp.seg0 + j] = LvEntry{q, (uint32_t)R, (uint32_t)V, 0u};
    if (R + cd.rows >= nv) break;  // the run covering the last row starts in this segment
    if (cd.state == 1) { set_err(err, ERR_LEVELS, lp.page); break; }
    if (cd.state != 0) { good = 0; break; }
    R += cd.rows;
    V += cd.valid;
    q = cd.exit;
  }
  if (!good)
    for (uint32_t j = 0; j < lp.nseg; ++j) ent[lp.seg0 + j].q = LV_NONE;
  ok[i] = good;
}

// The next run of a 1-bit hybrid stream for one lane (run_next's rules);
// byte(x) reads stream byte x (x < end).
template <class Byte>
__device__ __forceinline__ bool lv_run_next(const Byte& byte, uint64_t end, RunCur& c) {
  uint64_t pos = c.next;
  c.start += (int64_t)min(c.n, 1ull << 40);
  c.hp = pos;
  uint64_t h = 0;
  bool whole = false;
  for (int s = 0; s < 70; s += 7) {
    if (pos >= end) return false;
    const uint32_t b = byte(pos++);
    if (s == 63 && (b & 0x7e)) return false;
    h |= (uint64_t)(b & 0x7f) << s;
    if (!(b & 0x80)) { whole = true; break; }
  }
  if (!whole) return false;
  c.pay = pos;
  if (h & 1) {
    const uint64_t g = h >> 1;
    if (g > (1ull << 28) || g > end - pos) return false;
    c.bp = 1;
    c.n = g * 8;
    c.val = 0;
    c.next = pos + g;
  } else {
    if (pos >= end) return false;
    c.bp = 0;
    c.n = h >> 1;
    c.val = byte(pos);
    if (c.val > 1) return false;
    c.next = pos + 1;
  }
  return true;
}

// The whole level stream of one page by one wave (k_index's walk): tile
// entries, level checkpoints every LROWS rows, the non-null count.
__device__ void lv_page_walk(const LvStream& st, uint32_t p, uint32_t tile_begin, TileDev* tiles, uint32_t* ckl,
                             PageDev* pages, uint32_t* err, lds_u4* win) {
  WR r;
  r.init(st.base, st.lim, win);
  const bool lead = (threadIdx.x & 63) == 0;
  const uint64_t def_off = st.off, end = st.off + st.len;
  const int64_t nv = st.nv;
  RunCur c;
  c.next = def_off; c.start = 0; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0; c.hp = def_off;
  uint64_t before = 0;  // valid rows in runs before the current one
  bool have = false;
  TileDev td;
  for (int64_t target = 0; target < nv; target += LROWS) {
    while (!have || c.start + (int64_t)c.n <= target) {
      if (have) before += c.bp ? bp_popcount(r, c.pay, c.n) : (uint64_t)c.val * c.n;
      if (!run_next(r, end, 1, c) || (!c.bp && c.val > 1)) { set_err(err, ERR_LEVELS, p); return; }
      have = true;
    }
    const uint64_t skip = (uint64_t)(target - c.start);
    const uint32_t t = (uint32_t)(target / TILE_ROWS), sub = (uint32_t)((target % TILE_ROWS) / LROWS);
    if (sub == 0) {
      td.page = p;
      td.row0 = (uint32_t)target;
      td.k0 = (uint32_t)(before + (c.bp ? bp_popcount(r, c.pay, skip) : (uint64_t)c.val * skip));
      td.nn = 0;
      td.def_pos = (uint32_t)(c.hp - def_off);
      td.def_skip = (uint32_t)skip;
      td.val_pos = 0;
      td.val_skip = 0;
      if (lead) tiles[tile_begin + t] = td;
    }
    if (lead) ckl[(size_t)(tile_begin + t) * NLCK + sub] = make_lck(c, target, def_off + td.def_pos);
  }
  if (nv > 0 && lead)  // the last tile's checkpoints past the page's rows
    for (int64_t target = ((nv + LROWS - 1) / LROWS) * LROWS; target % TILE_ROWS != 0; target += LROWS)
      ckl[(size_t)(tile_begin + (uint32_t)(target / TILE_ROWS)) * NLCK + (target % TILE_ROWS) / LROWS] = LCK_NONE;
  if (nv > 0) {
    while (!have || c.start + (int64_t)c.n < nv) {
      if (have) before += c.bp ? bp_popcount(r, c.pay, c.n) : (uint64_t)c.val * c.n;
      if (!run_next(r, end, 1, c) || (!c.bp && c.val > 1)) { set_err(err, ERR_LEVELS, p); return; }
      have = true;
    }
    const uint64_t part = (uint64_t)(nv - c.start);
    const uint32_t nonnull = (uint32_t)(before + (c.bp ? bp_popcount(r, c.pay, part) : (uint64_t)c.val * part));
    if (lead) pages[p].nonnull = nonnull;
  }
}

// mode 0: one wave per linked segment; mode 1: one wave per page that could
// not be linked (lv_page_walk).  In mode 0 the segment and LV_XTRA bytes
// after it are staged in LDS; lanes read later bytes from memory.  Stream
// positions are relative to the level stream's start.
__global__ __launch_bounds__(64) void k_lv_tiles(const LvPage* lps, const uint32_t* seg_page, const LvEntry* ent,
                                                 const uint32_t* ok, PageDev* pages, const uint8_t* file,
                                                 const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim,
                                                 TileDev* tiles, uint32_t* ckl, uint32_t* err, int mode) {
  __shared__ __align__(16) uint8_t s_seg[LV_LDS];
  __shared__ uint32_t s_q[64], s_r[64], s_v[64];
  if (*(volatile uint32_t*)err != 0) return;
  if (mode == 1) {
    if (ok[blockIdx.x]) return;
    const uint32_t p = lps[blockIdx.x].page;
    const LvStream st = lv_stream(pages, p, file, scratch, file_lim, scratch_lim);
    lv_page_walk(st, p, pages[p].tile_begin, tiles, ckl, pages, err, (lds_u4*)&s_seg[0]);
    return;
  }
  const LvEntry e = ent[blockIdx.x];
  if (e.q == LV_NONE) return;
  const LvPage lp = lps[seg_page[blockIdx.x]];
  const uint32_t p = lp.page;
  const LvStream st = lv_stream(pages, p, file, scratch, file_lim, scratch_lim);
  const uint32_t tile_begin = pages[p].tile_begin;
  const uint32_t s0 = (blockIdx.x - lp.seg0) * LV_SEG;
  const uint32_t se = min(s0 + LV_SEG, st.len), sh = min(s0 + LV_SEG + LV_XTRA, st.len);
  const uint32_t d = lv_stage(st, s0, sh, &s_seg[0], 64);
  __syncthreads();
  const uint8_t* gbase = st.base + st.off;
  auto byte = [&](uint64_t x) -> uint32_t { return x < sh ? (uint32_t)s_seg[d + (uint32_t)x] : (uint32_t)gbase[x]; };
  const __attribute__((address_space(3))) uint32_t* w32 = (const __attribute__((address_space(3))) uint32_t*)&s_seg[0];
  // set bits among the k values of a bit-packed run from stream byte pay
  auto popc = [&](uint64_t pay, uint64_t k) -> uint64_t {
    uint64_t cnt = 0;
    if (pay + (k + 7) / 8 <= sh) {
      const uint32_t o = d + (uint32_t)pay;
      for (uint32_t i = 0; 8ull * i < k; i += 4) {
        uint32_t v = __builtin_amdgcn_alignbyte(w32[((o + i) >> 2) + 1], w32[(o + i) >> 2], (o + i) & 3);
        const uint64_t left = k - 8ull * i;
        if (left < 32) v &= (1u << left) - 1u;
        cnt += __popc(v);
      }
    } else {
      for (uint64_t i = 0; 8 * i < k; ++i) {
        uint32_t v = byte(pay + i);
        const uint64_t left = k - 8 * i;
        if (left < 8) v &= (1u << left) - 1u;
        cnt += __popc(v);
      }
    }
    return cnt;
  };
  auto pop = [&](const RunCur& c, uint64_t k) -> uint64_t { return c.bp ? popc(c.pay, k) : (uint64_t)c.val * k; };
  const int64_t nv = st.nv;
  const uint32_t lane = threadIdx.x;
  // lane 0: the first run header at or after each sub-segment's start, and
  // the rows before it; LV_NONE after the run covering the last row
  if (lane == 0) {
    RunCur c;
    c.next = e.q; c.start = (int64_t)e.rows; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0; c.hp = e.q;
    s_q[0] = e.q;
    s_r[0] = e.rows;
    uint32_t k = 1;
    bool done = false;
    for (;;) {
      const uint64_t h = done ? ~0ull : c.next;
      const int64_t rows = c.start + (int64_t)min(c.n, 1ull << 40);
      for (; k < 64 && h >= (uint64_t)s0 + (uint64_t)LV_SUB * k; ++k) {
        s_q[k] = h < se ? (uint32_t)h : LV_NONE;
        s_r[k] = (uint32_t)rows;
      }
      if (done || h >= se) break;
      if (!lv_run_next(byte, st.len, c)) {
        set_err(err, ERR_LEVELS, p);
        done = true;
        continue;
      }
      if (c.start + (int64_t)min(c.n, 1ull << 40) >= nv) done = true;
    }
    for (; k < 64; ++k) s_q[k] = LV_NONE;
  }
  __syncthreads();
  const uint64_t q0 = s_q[lane];
  const uint64_t qe = lane == 63 ? se : min((uint64_t)s0 + (uint64_t)LV_SUB * (lane + 1), (uint64_t)se);
  // valid rows of this lane's runs (up to the last row)
  uint64_t valid = 0;
  if (q0 != LV_NONE) {
    RunCur c;
    c.next = q0; c.start = (int64_t)s_r[lane]; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0; c.hp = q0;
    while (c.next < qe && lv_run_next(byte, st.len, c)) {
      const int64_t n = (int64_t)min(c.n, 1ull << 40);
      if (c.start + n >= nv) { valid += pop(c, (uint64_t)(nv - c.start)); break; }
      valid += pop(c, (uint64_t)n);
    }
  }
  s_v[lane] = (uint32_t)valid;
  __syncthreads();
  uint64_t before = e.valid;
  for (uint32_t k = 0; k < lane; ++k) before += s_v[k];
  if (q0 == LV_NONE) return;
  // this lane's runs once more: tile entries with their checkpoints
  RunCur c;
  c.next = q0; c.start = (int64_t)s_r[lane]; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0; c.hp = q0;
  while (c.next < qe && lv_run_next(byte, st.len, c)) {
    const int64_t lo = c.start, n = (int64_t)min(c.n, 1ull << 40), hi = min(lo + n, nv);
    for (int64_t t = (lo + TILE_ROWS - 1) / TILE_ROWS; t * TILE_ROWS < hi; ++t) {
      const uint64_t skip = (uint64_t)(t * TILE_ROWS - lo);
      TileDev td;
      td.page = p;
      td.row0 = (uint32_t)(t * TILE_ROWS);
      td.k0 = (uint32_t)(before + pop(c, skip));
      td.nn = 0;
      td.def_pos = (uint32_t)c.hp;
      td.def_skip = (uint32_t)skip;
      td.val_pos = 0;
      td.val_skip = 0;
      tiles[tile_begin + (uint32_t)t] = td;
      // the tile's level checkpoints, walking on from this run
      RunCur c2 = c;
      bool good = true;
      uint32_t* out = ckl + (size_t)(tile_begin + (uint32_t)t) * NLCK;
      for (int k = 0; k < NLCK; ++k) {
        const int64_t target = t * TILE_ROWS + (int64_t)k * LROWS;
        uint32_t lck = LCK_NONE;
        if (target < nv && good) {
          while (c2.start + (int64_t)min(c2.n, 1ull << 40) <= target)
            if (!lv_run_next(byte, st.len, c2)) { good = false; break; }
          if (good) lck = make_lck(c2, target, c.hp);
        }
        out[k] = lck;
      }
    }
    if (lo + n >= nv) {
      pages[p].nonnull = (uint32_t)(before + pop(c, (uint64_t)(nv - lo)));
      return;
    }
    before += pop(c, (uint64_t)n);
  }
}

// ---------------------------------------------------------------------------
// Long DELTA_BINARY_PACKED block chains.  A block is a ULEB128 zigzag
// minimum delta, M miniblock bit widths (a byte each) and the miniblocks'
// packed deltas, so its size follows from its header, and the blocks form a
// chain from the stream's block 0.  As for level streams: k_dl_cand walks
// DL_CAND candidate chains per DL_SEG-byte segment (every block taken as a
// full block), k_dl_link follows the true chain through them, k_dl_fill
// walks each segment's blocks from its entry -- exactly, the last block
// holding only the miniblocks its values use -- storing every block's
// position and, after the last block, the stream's end (or walks a page
// whole when its chain cannot be linked, mode 1), and k_dl_tiles gives each
// tile its entry block and block checkpoints from the stored positions.
// ---------------------------------------------------------------------------
constexpr uint32_t DL_LDS = DL_SEG + 64;
static_assert(DL_CAND <= DL_SEG && DL_CAND % 64 == 0, "candidates: whole waves inside a segment");

struct DlStream {
  const uint8_t* base;
  uint64_t lim;       // readable bytes of base (a multiple of 16)
  uint64_t off;       // value-stream offset in base
  uint32_t len;       // value-stream bytes
  uint32_t at;        // stream offset of block 0
  uint32_t B, M, per; // values per block, miniblocks per block, values per miniblock
  uint64_t total;     // values in the stream (the page's non-null count)
  uint64_t nblocks;   // blocks: value 0 is in the stream header
};
__device__ __forceinline__ DlStream dl_stream(const PageDev* pages, uint32_t p, const uint8_t* file,
                                              const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim) {
  DlStream st;
  const bool sc = (pages[p].flags & 2) != 0;
  st.base = sc ? scratch : file;
  st.lim = sc ? scratch_lim : file_lim;
  st.off = pages[p].val_off;
  st.len = pages[p].val_len;
  st.at = pages[p].blocks_at;
  st.B = pages[p].enc_w;
  st.M = pages[p].enc_m;
  st.per = st.M ? st.B / st.M : 0;
  st.total = pages[p].nonnull;
  st.nblocks = (st.total > 1 && st.B) ? (st.total - 1 + st.B - 1) / st.B : 0;
  return st;
}

// One workgroup of DL_CAND lanes per segment; the segment and the longest
// block header after it are staged in LDS.
__global__ __launch_bounds__(DL_CAND) void k_dl_cand(const DlPage* dps, const uint32_t* seg_page, const PageDev* pages,
                                                     const uint8_t* file, const uint8_t* scratch, uint64_t file_lim,
                                                     uint64_t scratch_lim, DlCand* cand, const uint32_t* err) {
  __shared__ __align__(16) uint8_t s_seg[DL_LDS];
  const uint32_t sg = blockIdx.x, c = threadIdx.x;
  DlCand out = {0u, 0u, 1u, 0u};
  if (*(const volatile uint32_t*)err == 0) {
    const DlPage dp = dps[seg_page[sg]];
    const DlStream st = dl_stream(pages, dp.page, file, scratch, file_lim, scratch_lim);
    const uint64_t s0 = (uint64_t)st.at + (uint64_t)(sg - dp.seg0) * DL_SEG;
    out.exit = (uint32_t)(s0 + c);
    if (s0 < st.len) {
      const uint32_t se = (uint32_t)min(s0 + DL_SEG, (uint64_t)st.len);       // block headers of this segment: [s0, se)
      const uint32_t sh = (uint32_t)min(s0 + DL_SEG + 32, (uint64_t)st.len);  // staged: [s0, sh)
      const uint64_t g0 = st.off + s0, a0 = g0 & ~15ull, ga = st.off + sh;
      for (uint32_t k = c; a0 + 16ull * k < ga; k += DL_CAND) {
        const uint64_t a = a0 + 16ull * k;
        wr_u4 v = {0u, 0u, 0u, 0u};
        if (a + 16 <= st.lim) v = *reinterpret_cast<const wr_u4*>(st.base + a);
        *(lds_u4*)(&s_seg[16 * k]) = v;
      }
      __syncthreads();
      const uint32_t d = (uint32_t)(g0 - a0) - (uint32_t)s0;  // LDS offset of stream byte x: d + x
      uint32_t q = (uint32_t)s0 + c, count = 0, state = 0;
      while (q < se) {
        uint32_t x = q;
        bool whole = false;
        for (uint32_t b7 = 0; b7 < 70; b7 += 7) {  // minimum delta (a header a block of 10 bytes at most)
          if (x >= st.len) break;
          const uint32_t b = s_seg[d + x];
          ++x;
          if (b7 == 63 && (b & 0x7e)) break;
          if (!(b & 0x80)) { whole = true; break; }
        }
        if (!whole || st.M > st.len - x) { state = 1; break; }
        uint64_t body = 0;
        bool bad = false;
        for (uint32_t m = 0; m < st.M; ++m) {
          const uint32_t w = s_seg[d + x + m];
          bad |= w > dp.maxw;
          body += (uint64_t)st.per * w / 8;
        }
        x += st.M;
        if (bad || body > st.len - x) { state = 1; break; }
        q = x + (uint32_t)body;
        ++count;
      }
      out = DlCand{q, count, state, 0u};
    }
  }
  cand[(size_t)sg * DL_CAND + c] = out;
}

// One thread per page (see k_lv_link): ent[segment] = (entry offset, block
// index) along the true chain, up to the segment of the last block.
__global__ void k_dl_link(const DlPage* dps, int npg, PageDev* pages, const DlCand* cand, DlEntry* ent, uint32_t* ok,
                          uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npg) return;
  const DlPage dp = dps[i];
  for (uint32_t j = 0; j < dp.nseg; ++j) ent[dp.seg0 + j].q = LV_NONE;
  ok[i] = 1;
  if (*(volatile uint32_t*)err != 0) return;
  const DlStream st = dl_stream(pages, dp.page, nullptr, nullptr, 0, 0);
  if (st.nblocks == 0) {
    pages[dp.page].chars_at = st.at;
    return;
  }
  uint32_t q = st.at, good = 1;
  uint64_t k = 0;
  for (;;) {
    if (q >= st.len) { set_err(err, ERR_DELTA, dp.page); break; }  // the stream ends before the last block
    const uint32_t j = (q - st.at) / DL_SEG, c = (q - st.at) % DL_SEG;
    if (j >= dp.nseg || c >= DL_CAND) { good = 0; break; }
    const DlCand cd = cand[(size_t)(dp.seg0 + j) * DL_CAND + c];
    ent[dp.seg0 + j] = DlEntry{q, (uint32_t)k};
    if (k + cd.count >= st.nblocks) break;  // the last block starts in this segment
    if (cd.state != 0) {
      if (k + cd.count + 1 == st.nblocks) break;  // at the last block, which need not be full
      set_err(err, ERR_DELTA, dp.page);
      break;
    }
    k += cd.count;
    q = cd.exit;
  }
  if (!good) {
    for (uint32_t j = 0; j < dp.nseg; ++j) ent[dp.seg0 + j].q = LV_NONE;
    ok[i] = 0;
  }
}

// mode 0: one wave per segment, from its entry, over the blocks whose header
// lies in it; mode 1: one wave per page that could not be linked.
__global__ __launch_bounds__(64) void k_dl_fill(const DlPage* dps, const uint32_t* seg_page, const DlEntry* ent,
                                                const uint32_t* ok, PageDev* pages, const uint8_t* file,
                                                const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim,
                                                uint32_t* blkpos, uint32_t* err, int mode) {
  __shared__ wr_u4 s_win[WIN / 16];
  if (*(volatile uint32_t*)err != 0) return;
  uint32_t di, q, seg_end;
  uint64_t k;
  if (mode == 0) {
    const DlEntry e = ent[blockIdx.x];
    if (e.q == LV_NONE) return;
    di = seg_page[blockIdx.x];
    q = e.q;
    k = e.k;
    seg_end = pages[dps[di].page].blocks_at + (blockIdx.x - dps[di].seg0 + 1) * DL_SEG;
  } else {
    di = blockIdx.x;
    if (ok[di]) return;
    q = pages[dps[di].page].blocks_at;
    k = 0;
    seg_end = 0xffffffffu;
  }
  const DlPage dp = dps[di];
  const DlStream st = dl_stream(pages, dp.page, file, scratch, file_lim, scratch_lim);
  const bool lead = threadIdx.x == 0;
  WR r;
  r.init(st.base, st.lim, (lds_u4*)&s_win[0]);
  const uint64_t vend = st.off + st.len;
  uint64_t qa = st.off + q;
  for (; k < st.nblocks && qa - st.off < seg_end; ++k) {
    if (lead) blkpos[dp.blk0 + k] = (uint32_t)(qa - st.off);
    bool bad = false;
    br_uleb(r, qa, vend, bad);  // minimum delta
    if (bad || st.M > vend - qa) { set_err(err, ERR_DELTA, dp.page); return; }
    const uint64_t left = st.total - 1 - k * st.B;  // values from this block on
    const uint64_t used = left < st.B ? left : st.B;
    const uint64_t used_mb = (used + st.per - 1) / st.per;
    uint64_t body = 0;
    for (uint64_t m = 0; m < used_mb; ++m) {
      const uint32_t w = r.byte(qa + m);
      if (w > dp.maxw) { set_err(err, ERR_DELTA, dp.page); return; }
      body += (uint64_t)st.per * w / 8;
    }
    qa += st.M;
    if (body > vend - qa) { set_err(err, ERR_DELTA, dp.page); return; }
    qa += body;
  }
  if (k == st.nblocks && lead) pages[dp.page].chars_at = (uint32_t)(qa - st.off);
}

// One thread per tile of the pages above: the block holding the tile's
// first delta is its entry; blocks from there to the one holding its last
// delta are its checkpoints.  Tiles that need no block keep the entry the
// index pass gave them (block 0, no checkpoints).
__global__ void k_dl_tiles(const DlPage* dps, const uint32_t* tile_dp, int ntl, const PageDev* pages, TileDev* tiles,
                           Ck* ckv, const uint32_t* blkpos, const uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntl || *(const volatile uint32_t*)err != 0) return;
  const DlPage dp = dps[tile_dp[i]];
  const uint32_t T = pages[dp.page].tile_begin + ((uint32_t)i - dp.tl0);
  const uint64_t B = pages[dp.page].enc_w;
  const uint64_t k0 = tiles[T].k0, nn = tiles[T].nn;
  if (nn == 0 || k0 + nn <= 1) return;
  const uint64_t first = k0 == 0 ? 1 : k0;
  const uint64_t bu = (first - 1) / B, lastb = (k0 + nn - 2) / B;
  const uint32_t vp = blkpos[dp.blk0 + bu];
  tiles[T].val_pos = vp;
  tiles[T].val_skip = (uint32_t)((first - 1) % B);
  for (uint64_t b = bu; b <= lastb && b - bu < (uint64_t)NSUB; ++b)
    ckv[(size_t)T * NSUB + (b - bu)] = ck_at((uint64_t)(blkpos[dp.blk0 + b] - vp));
}

// ---------------------------------------------------------------------------
// Long dictionary-index streams: hybrid runs of width w after the width
// byte.  Same scheme once more: k_di_cand walks di_cand(w) candidate chains
// per DI_SEG-byte segment counting values, k_di_link follows the true chain
// up to the run covering the page's last non-null value, k_di_fill walks
// each segment's runs from its entry and gives the tiles whose first value
// lies in them their entry run (or walks a page whole, mode 1), and
// k_di_ckpt derives each tile's value checkpoints from its entry, one per
// lane, four tiles per wave.
// ---------------------------------------------------------------------------
constexpr uint32_t DI_LDS = DI_SEG + 64;
constexpr uint32_t DI_WG = 256;

struct DiStream {
  const uint8_t* base;
  uint64_t lim, off;  // value stream at base + off
  uint32_t len;       // value-stream bytes
  uint32_t w;         // index bit width
  uint64_t total;     // indices (the page's non-null count)
};
__device__ __forceinline__ DiStream di_stream(const PageDev* pages, uint32_t p, const uint8_t* file,
                                              const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim) {
  DiStream st;
  const bool sc = (pages[p].flags & 2) != 0;
  st.base = sc ? scratch : file;
  st.lim = sc ? scratch_lim : file_lim;
  st.off = pages[p].val_off;
  st.len = pages[p].val_len;
  st.w = pages[p].enc_w;
  st.total = pages[p].nonnull;
  return st;
}

// One workgroup of DI_WG lanes per segment, each lane walking every
// DI_WG-th candidate; the segment's run headers are staged in LDS.
// Segment sg's candidates are cand[sg DI_CAND_MAX ..], di_cand(w) of them.
// Chains that reach the same run header past the candidates' start bytes go
// on alike, so each such header is walked on from once (by the first
// candidate that reached it, found through an LDS table over the DI_DEDUP
// bytes that follow the start bytes).
constexpr uint32_t DI_PER = DI_CAND_MAX / DI_WG;
constexpr uint32_t DI_DEDUP = 2048;

__global__ __launch_bounds__(DI_WG) void k_di_cand(const DiPage* dps, const uint32_t* seg_page, const PageDev* pages,
                                                   const uint8_t* file, const uint8_t* scratch, uint64_t file_lim,
                                                   uint64_t scratch_lim, DiCand* cand, const uint32_t* err) {
  __shared__ __align__(16) uint8_t s_seg[DI_LDS];
  __shared__ uint32_t s_first[DI_DEDUP], s_exit[DI_CAND_MAX], s_cnt[DI_CAND_MAX];
  if (*(const volatile uint32_t*)err != 0) return;
  const uint32_t sg = blockIdx.x;
  const DiPage dp = dps[seg_page[sg]];
  const DiStream st = di_stream(pages, dp.page, file, scratch, file_lim, scratch_lim);
  const uint32_t j = sg - dp.seg0;
  const uint64_t s0 = 1 + (uint64_t)j * DI_SEG;  // runs start after the width byte
  DiCand* out = cand + (size_t)sg * DI_CAND_MAX;
  const uint32_t ncand = di_cand(st.w);
  if (s0 >= st.len) {
    for (uint32_t c = threadIdx.x; c < ncand; c += DI_WG) out[c] = DiCand{DI_BAD, 0u};
    return;
  }
  const uint32_t se = (uint32_t)min(s0 + DI_SEG, (uint64_t)st.len);       // run headers of this segment: [s0, se)
  const uint32_t sh = (uint32_t)min(s0 + DI_SEG + 16, (uint64_t)st.len);  // staged: [s0, sh)
  const uint64_t g0 = st.off + s0, a0 = g0 & ~15ull, ga = st.off + sh;
  for (uint32_t k = threadIdx.x; a0 + 16ull * k < ga; k += DI_WG) {
    const uint64_t a = a0 + 16ull * k;
    wr_u4 v = {0u, 0u, 0u, 0u};
    if (a + 16 <= st.lim) v = *reinterpret_cast<const wr_u4*>(st.base + a);
    *(lds_u4*)(&s_seg[16 * k]) = v;
  }
  for (uint32_t k = threadIdx.x; k < DI_DEDUP; k += DI_WG) s_first[k] = 0xffffffffu;
  __syncthreads();
  const uint32_t d = (uint32_t)(g0 - a0) - (uint32_t)s0;  // LDS offset of stream byte x: d + x
  const uint32_t vb = (st.w + 7) / 8;
  // walks the runs whose header lies before lim from q, counting values;
  // false at an invalid run
  const __attribute__((address_space(3))) uint32_t* w32 = (const __attribute__((address_space(3))) uint32_t*)&s_seg[0];
  auto walk = [&](uint32_t& q, uint32_t lim, uint32_t& count) -> bool {
    while (q < lim) {
      uint64_t h = 0;
      uint32_t x = q, hl = 0;
      if (q + 8 <= sh) {  // the common short header, from one dword
        const uint32_t o = d + q;
        uint32_t h32 = 0;
        hl = uleb4(__builtin_amdgcn_alignbyte(w32[(o >> 2) + 1], w32[o >> 2], o & 3), h32);
        h = h32;
        x = q + hl;
      }
      if (hl == 0) {
        bool whole = false;
        for (uint32_t b7 = 0; b7 < 70; b7 += 7) {  // a header is 10 bytes at most
          if (x >= st.len) break;
          const uint32_t b = s_seg[d + x];
          ++x;
          if (b7 == 63 && (b & 0x7e)) break;
          h |= (uint64_t)(b & 0x7f) << b7;
          if (!(b & 0x80)) { whole = true; break; }
        }
        if (!whole) return false;
      }
      uint64_t n, nb;
      if (h & 1) {
        n = (h >> 1) * 8;
        nb = (h >> 1) * st.w;
        if ((h >> 1) > (1ull << 28) || nb > st.len - x) return false;
      } else {
        n = h >> 1;
        nb = vb;
        if (nb > st.len - x) return false;
      }
      count = lv_sat(count, n);
      q = x + (uint32_t)nb;
    }
    return true;
  };
  const uint32_t wend = (uint32_t)min(s0 + ncand, (uint64_t)se);  // end of the start bytes
  uint32_t qa[DI_PER], ca[DI_PER];
  bool oka[DI_PER];
#pragma unroll
  for (uint32_t u = 0; u < DI_PER; ++u) {
    const uint32_t c = threadIdx.x + u * DI_WG;
    qa[u] = (uint32_t)s0 + c;
    ca[u] = 0;
    oka[u] = false;
    if (c < ncand) {
      oka[u] = walk(qa[u], wend, ca[u]);
      if (oka[u] && qa[u] < se && qa[u] - wend < DI_DEDUP) atomicMin(&s_first[qa[u] - wend], c);
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t u = 0; u < DI_PER; ++u) {
    const uint32_t c = threadIdx.x + u * DI_WG;
    if (c < ncand && oka[u] && qa[u] < se) {
      const uint32_t lead = qa[u] - wend < DI_DEDUP ? s_first[qa[u] - wend] : c;
      if (lead == c) {
        uint32_t q2 = qa[u], c2 = 0;
        s_exit[c] = walk(q2, se, c2) ? q2 : DI_BAD;
        s_cnt[c] = c2;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t u = 0; u < DI_PER; ++u) {
    const uint32_t c = threadIdx.x + u * DI_WG;
    if (c >= ncand) continue;
    DiCand r = DiCand{oka[u] ? qa[u] : DI_BAD, ca[u]};
    if (oka[u] && qa[u] < se) {
      const uint32_t lead = qa[u] - wend < DI_DEDUP ? s_first[qa[u] - wend] : c;
      r = DiCand{s_exit[lead], lv_sat(ca[u], s_cnt[lead])};
    }
    out[c] = r;
  }
}

// One thread per page (see k_lv_link): ent[segment] = (entry offset, index
// of the entry run's first value) along the true chain.
__global__ void k_di_link(const DiPage* dps, int npg, const PageDev* pages, const DiCand* cand, DlEntry* ent,
                          uint32_t* ok, uint32_t* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npg) return;
  const DiPage dp = dps[i];
  for (uint32_t j = 0; j < dp.nseg; ++j) ent[dp.seg0 + j].q = LV_NONE;
  ok[i] = 1;
  if (*(volatile uint32_t*)err != 0) return;
  const DiStream st = di_stream(pages, dp.page, nullptr, nullptr, 0, 0);
  if (st.total == 0) return;
  uint32_t q = 1, good = 1;
  uint64_t K = 0;
  for (;;) {
    if (q >= st.len) { set_err(err, ERR_VALUES, dp.page); break; }  // the runs end before the last value
    const uint32_t j = (q - 1) / DI_SEG, c = (q - 1) % DI_SEG;
    if (j >= dp.nseg || c >= di_cand(st.w)) { good = 0; break; }
    const DiCand cd = cand[(size_t)(dp.seg0 + j) * DI_CAND_MAX + c];
    ent[dp.seg0 + j] = DlEntry{q, (uint32_t)K};
    if (K + cd.count >= st.total) break;  // the run covering the last value starts in this segment
    if (cd.exit == DI_BAD) { set_err(err, ERR_VALUES, dp.page); break; }
    K += cd.count;
    q = cd.exit;
  }
  if (!good) {
    for (uint32_t j = 0; j < dp.nseg; ++j) ent[dp.seg0 + j].q = LV_NONE;
    ok[i] = 0;
  }
}

// mode 0: one wave per segment, from its entry; mode 1: one wave per page
// that could not be linked.  Tiles holding values get the run that holds
// their first value as entry.
__global__ __launch_bounds__(64) void k_di_fill(const DiPage* dps, const uint32_t* seg_page, const DlEntry* ent,
                                                const uint32_t* ok, const PageDev* pages, const uint8_t* file,
                                                const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim,
                                                TileDev* tiles, uint32_t* err, int mode) {
  __shared__ wr_u4 s_win[WIN / 16];
  if (*(volatile uint32_t*)err != 0) return;
  uint32_t di, q, seg_end;
  uint64_t K;
  if (mode == 0) {
    const DlEntry e = ent[blockIdx.x];
    if (e.q == LV_NONE) return;
    di = seg_page[blockIdx.x];
    q = e.q;
    K = e.k;
    seg_end = 1 + (blockIdx.x - dps[di].seg0 + 1) * DI_SEG;
  } else {
    di = blockIdx.x;
    if (ok[di] || pages[dps[di].page].nonnull == 0) return;
    q = 1;
    K = 0;
    seg_end = 0xffffffffu;
  }
  const DiPage dp = dps[di];
  const DiStream st = di_stream(pages, dp.page, file, scratch, file_lim, scratch_lim);
  const uint32_t tb = pages[dp.page].tile_begin;
  const uint32_t nt = (uint32_t)(((uint64_t)pages[dp.page].num_values + TILE_ROWS - 1) / TILE_ROWS);
  // first tile whose first value is at or after K (k0 does not decrease)
  uint32_t lo_t = 0, hi_t = nt;
  while (lo_t < hi_t) {
    const uint32_t mid = (lo_t + hi_t) / 2;
    if (tiles[tb + mid].k0 < K) lo_t = mid + 1; else hi_t = mid;
  }
  uint32_t t = lo_t;
  const bool lead = threadIdx.x == 0;
  WR r;
  r.init(st.base, st.lim, (lds_u4*)&s_win[0]);
  const uint64_t vend = st.off + st.len;
  RunCur c;
  c.next = st.off + q; c.start = (int64_t)K; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0; c.hp = c.next;
  for (;;) {
    if (c.next - st.off >= seg_end) return;  // the next run belongs to a later segment
    if (!run_next(r, vend, st.w, c)) { set_err(err, ERR_VALUES, dp.page); return; }
    const uint64_t lo = (uint64_t)c.start, hi = lo + min(c.n, 1ull << 40);
    for (; t < nt; ++t) {
      const uint32_t k0 = tiles[tb + t].k0, nn = tiles[tb + t].nn;
      if (k0 >= hi) break;
      if (nn > 0 && lead) {
        tiles[tb + t].val_pos = (uint32_t)(c.hp - st.off);
        tiles[tb + t].val_skip = (uint32_t)(k0 - lo);
      }
    }
    if (hi >= st.total) return;
  }
}

// A dictionary-index run for one lane (run_next's rules for width w; the
// RLE value is not read); byte(x) reads stream byte x (x < end).
template <class Byte>
__device__ __forceinline__ bool di_run_next(const Byte& byte, uint64_t end, uint32_t w, RunCur& c) {
  uint64_t pos = c.next;
  c.start += (int64_t)min(c.n, 1ull << 40);
  c.hp = pos;
  uint64_t h = 0;
  bool whole = false;
  for (int s = 0; s < 70; s += 7) {
    if (pos >= end) return false;
    const uint32_t b = byte(pos++);
    if (s == 63 && (b & 0x7e)) return false;
    h |= (uint64_t)(b & 0x7f) << s;
    if (!(b & 0x80)) { whole = true; break; }
  }
  if (!whole) return false;
  c.pay = pos;
  c.val = 0;
  if (h & 1) {
    const uint64_t g = h >> 1;
    if (g > (1ull << 28) || g * w > end - pos) return false;
    c.bp = 1;
    c.n = g * 8;
    c.next = pos + g * w;
  } else {
    const uint32_t vb = (w + 7) / 8;
    if (vb > end - pos) return false;
    c.bp = 0;
    c.n = h >> 1;
    c.next = pos + vb;
  }
  return true;
}

// Four tiles per wave, lane 16 i + s computing checkpoint s of tile i: the
// state of the run holding value k0 + 64 s, reached by walking the runs
// from the tile's entry.
__global__ __launch_bounds__(64) void k_di_ckpt(const DiPage* dps, const uint32_t* tile_dp, int ntl,
                                                const PageDev* pages, const TileDev* tiles, const uint8_t* file,
                                                const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim,
                                                Ck* ckv, const uint32_t* err) {
  static_assert(NSUB == 16, "16 lanes per tile");
  if (*(const volatile uint32_t*)err != 0) return;
  const uint32_t i = blockIdx.x * 4 + threadIdx.x / 16, sub = threadIdx.x % 16;
  if ((int)i >= ntl) return;
  const DiPage dp = dps[tile_dp[i]];
  const DiStream st = di_stream(pages, dp.page, file, scratch, file_lim, scratch_lim);
  const uint32_t T = pages[dp.page].tile_begin + (i - dp.tl0);
  const TileDev td = tiles[T];
  if ((uint64_t)sub * SUB_ROWS >= td.nn) return;
  const uint64_t entry = st.off + td.val_pos, end = st.off + st.len;
  const uint8_t* base = st.base;
  auto byte = [&](uint64_t x) -> uint32_t { return base[x]; };
  const int64_t target = (int64_t)td.k0 + (int64_t)sub * SUB_ROWS;
  RunCur c;
  c.next = entry; c.start = (int64_t)td.k0 - (int64_t)td.val_skip; c.n = 0; c.bp = 0; c.val = 0; c.pay = 0;
  c.hp = entry;
  do {
    if (!di_run_next(byte, end, st.w, c)) return;  // not reached for a linked stream
  } while (c.start + (int64_t)min(c.n, 1ull << 40) <= target);
  ckv[(size_t)T * NSUB + sub] = make_ck(c, target, st.w, entry, false);
}

}  // namespace pqk
