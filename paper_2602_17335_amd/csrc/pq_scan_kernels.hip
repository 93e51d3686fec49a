// pq_scan_kernels.hip -- kernels of one scan (everything pq_scan enqueues),
// and k_prepass, which pq_open_device runs once to build the tile prefix.
//
//   k_snappy        Snappy page bodies -> workspace (one wave per page)
//   k_dba           DELTA_BYTE_ARRAY pages -> PLAIN layout (one wave per page)
//   k_snap_index    Snappy block index and element counts (at open, one wave per page)
//   k_snap_order    a scan's Snappy blocks in buckets of element count
//   k_snappy_blk    Snappy page bodies with a block index (one lane per 64 KiB block,
//                   SNAP_LANES blocks per wave, elements in batches)
//   k_prep          validity edge words cleared / REQUIRED validity set to ones
//   k_dict          dictionary pages -> device dictionaries
//   k_prepass       per-tile DELTA sums and string byte counts (at open)
//   k_str_total     offsets[rows] and the chars capacity check of string columns
//   k_decode_fixed  definition levels; PLAIN / dictionary INT32, INT64, DOUBLE values
//   k_decode_delta  definition levels; DELTA_BINARY_PACKED INT32 / INT64 values
//   k_decode_str    definition levels; PLAIN / dictionary BYTE_ARRAY values -> offsets and chars
//
// The tile prefix (one uint64 per tile of the file, plus one) is the
// exclusive prefix sum, in file tile order, of each tile's DELTA sum or
// string byte count (0 for other tiles).  A DELTA tile's carry is the
// difference of the prefix at the tile and at its page's first tile; a
// string tile's chars start is the difference at the tile and at the scan's
// first tile of the column.  Both are exact modulo 2^64.
//
// Work unit of the prepass and decode kernels: one TILE_ROWS-row tile
// of one page per wave, four independent tiles per 256-thread workgroup, no
// workgroup barriers.  A tile is entered through the index built at open:
// besides the tile's own entry points, the run header holding every SUB_ROWS-th
// row of the level stream, every SUB_ROWS-th value of a dictionary-index
// stream, and every block header of a DELTA stream are recorded.  Lane l
// decodes rows (or values) [16 l, 16 l + 16) starting from the nearest such
// checkpoint, so no lane follows the chain of run headers from the tile's
// start.  Rows are then assigned lane-interleaved (row 64 i + l) so that every
// output store of a wave is one contiguous 256- or 512-byte range.
#include <hip/hip_runtime.h>

#include "pq_device.hpp"
#include "pq_internal.h"

namespace pqk {

constexpr int WG = 256;
constexpr int NWAVES = WG / 64;
constexpr int TR = TILE_ROWS;         // rows per tile
constexpr int LPER = TR / 64;         // rows (or values) decoded per lane
constexpr int NWORDS = TR / 32;       // validity words per tile
constexpr int NGROUPS = TR / 64;      // 64-row groups per tile
constexpr int PADN = TR + TR / 16 + 4;  // padded per-wave LDS arrays (see pad())
constexpr int GROUP_CHARS = 3072;     // per-wave LDS bytes for one 64-row group of strings
static_assert(SUB_ROWS == 4 * LPER, "four lanes share one sub-tile checkpoint");
static_assert(LROWS == LPER, "one level checkpoint per lane");
static_assert(NWORDS == 32, "lane j < 32 holds validity word j");

// Per-wave LDS arrays written lane-blocked (lane l writes entries 16 l ..)
// and read lane-interleaved: one spare slot every 16 entries keeps both
// patterns free of bank conflicts.
__device__ __forceinline__ uint32_t pad(uint32_t j) { return j + (j >> 4); }

// Wave-uniform reads of tables that no kernel of a scan writes (the column
// table, the file's page table, tile index, dictionaries and tile prefix).
// Every lane reads the same address; the value is then moved dword by dword
// into scalar registers, so that it does not hold vector registers for the
// rest of the tile (the compiler cannot prove these tables unwritten and so
// would keep a vector load's result in VGPRs).
template <class T>
__device__ __forceinline__ T sload(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized tables");
  const T v = *p;
  T r;
  const uint32_t* a = reinterpret_cast<const uint32_t*>(&v);
  uint32_t* b = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
  for (uint32_t i = 0; i < sizeof(T) / 4; ++i) b[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)a[i]);
  return r;
}

struct Streams {
  const uint8_t* dbase;
  uint64_t doff, dend;
  const uint8_t* vbase;
  uint64_t voff, vend;
};

__device__ __forceinline__ Streams page_streams(const PageDev& pg, const ColScan& cs, uint8_t* ws) {
  const uint8_t* file = cs.fd.file;
  Streams s;
  const uint8_t* sb = ws + cs.ws_scratch;
  if (pg.flags & 1) { s.dbase = sb; s.doff = pg.def_off - cs.scratch_base; }
  else { s.dbase = file; s.doff = pg.def_off; }
  s.dend = s.doff + (uint64_t)pg.def_len;
  if (pg.flags & 4) { s.vbase = ws + cs.ws_xscratch; s.voff = pg.val_off - cs.xscratch_base; }
  else if (pg.flags & 2) { s.vbase = sb; s.voff = pg.val_off - cs.scratch_base; }
  else { s.vbase = file; s.voff = pg.val_off; }
  s.vend = s.voff + pg.val_len;
  return s;
}

// ---------------------------------------------------------------------------
// global byte source: bytes [origin, origin + len) of a 16-byte aligned base.
// Reads are aligned dwords, so a read near the end may touch up to 12 bytes
// past `len`; every stream lies inside the file (followed by at least its
// footer) or inside a decompressed region (followed by SCRATCH_PAD bytes).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(1))) const uint8_t glb_u8;
typedef __attribute__((address_space(1))) const uint32_t glb_u32;
typedef __attribute__((address_space(1))) const uint64_t glb_u64;

template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

typedef uint32_t u32x4w __attribute__((ext_vector_type(4), aligned(4)));  // 16 bytes at a dword address
typedef const __attribute__((address_space(1))) u32x4w glb_u32x4w;

struct GSrc {
  using P = uint64_t;  // stream positions (bytes, bits)
  using I = int64_t;   // value numbers
  glb_u8* base;
  uint64_t origin;  // absolute offset of position 0
  uint64_t len;
  // bytes p .. p+7
  __device__ __forceinline__ uint64_t window(uint64_t p) const { return bits(p * 8, 64); }
  __device__ __forceinline__ uint64_t bits64(uint64_t bit, uint32_t w) const { return bits(bit, w); }
  __device__ __forceinline__ uint32_t byte(uint64_t i) const { return i < len ? (uint32_t)base[origin + i] : 0u; }
  // w (<= 64) bits at bit position `bit`
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
  // the 4 dwords from the one holding bit `bit` (16 bytes: reads at most 15
  // past the bit's byte); s receives the bit's offset in the first
  __device__ __forceinline__ u32x4w quad(uint64_t bit, uint32_t& s) const {
    const uint64_t b = origin * 8 + bit;
    s = (uint32_t)(b & 31);
    return *(glb_u32x4w*)(reinterpret_cast<glb_u32*>(base) + (b >> 5));
  }
  // little-endian u32 / u64 at byte position pos: aligned dwords joined with
  // byte funnel shifts (no data-dependent branch, so a wave issues all its
  // loads before the first wait)
  __device__ __forceinline__ uint32_t u32(uint64_t pos) const {
    const uint64_t a = origin + pos;
    glb_u32* q = reinterpret_cast<glb_u32*>(base + (a & ~3ull));
    return __builtin_amdgcn_alignbyte(q[1], q[0], (uint32_t)(a & 3));
  }
  __device__ __forceinline__ uint64_t u64(uint64_t pos) const {
    const uint64_t a = origin + pos;
    glb_u32* q = reinterpret_cast<glb_u32*>(base + (a & ~3ull));
    const uint32_t q0 = q[0], q1 = q[1], q2 = q[2], sh = (uint32_t)(a & 3);
    return (uint64_t)__builtin_amdgcn_alignbyte(q1, q0, sh) | ((uint64_t)__builtin_amdgcn_alignbyte(q2, q1, sh) << 32);
  }
};

__device__ __forceinline__ GSrc gsrc(const uint8_t* base, uint64_t a0, uint64_t a1) {
  GSrc s;
  s.base = (glb_u8*)base;
  s.origin = a0;
  s.len = a1 > a0 ? a1 - a0 : 0;
  return s;
}

// The same stream with 32-bit positions, for streams shorter than NARROW_LEN
// bytes of pages with fewer than NARROW_VALUES values (every bit position and
// every value number of the walks below then fits 31 bits).  The base is the
// dword holding stream byte 0 (wave-uniform), so loads take a 32-bit offset.
constexpr uint32_t NARROW_LEN = 1u << 28;
constexpr uint32_t NARROW_VALUES = 1u << 29;
struct GSrc32 {
  using P = uint32_t;
  using I = int32_t;
  glb_u32* abase;
  uint32_t m;    // stream byte 0 is byte m of abase[0]
  uint32_t len;
  __device__ __forceinline__ uint32_t byte(uint32_t i) const {
    const uint32_t a = i + m;
    return i < len ? (abase[a >> 2] >> (8 * (a & 3))) & 0xffu : 0u;
  }
  // w (<= 32) bits at bit position `bit`
  __device__ __forceinline__ uint32_t bits(uint32_t bit, uint32_t w) const {
    const uint32_t b = bit + 8 * m;
    const uint32_t d = b >> 5;
    const uint32_t v = __builtin_amdgcn_alignbit(abase[d + 1], abase[d], b & 31);
    return v & (w >= 32 ? 0xffffffffu : ((1u << w) - 1u));
  }
  __device__ __forceinline__ u32x4w quad(uint32_t bit, uint32_t& s) const {
    const uint32_t b = bit + 8 * m;
    s = b & 31;
    return *(glb_u32x4w*)(abase + (b >> 5));
  }
  // w (<= 64) bits at bit position `bit`
  __device__ __forceinline__ uint64_t bits64(uint32_t bit, uint32_t w) const {
    const uint32_t b = bit + 8 * m;
    const uint32_t d = b >> 5, sh = b & 31;
    const uint32_t q0 = abase[d], q1 = abase[d + 1], q2 = abase[d + 2];
    const uint64_t v = (uint64_t)__builtin_amdgcn_alignbit(q1, q0, sh) |
                       ((uint64_t)__builtin_amdgcn_alignbit(q2, q1, sh) << 32);
    return w >= 64 ? v : (v & ((1ull << w) - 1));
  }
  __device__ __forceinline__ uint64_t window(uint32_t p) const {
    const uint32_t a = p + m, d = a >> 2, sh = a & 3;
    const uint32_t q0 = abase[d], q1 = abase[d + 1], q2 = abase[d + 2];
    return (uint64_t)__builtin_amdgcn_alignbyte(q1, q0, sh) | ((uint64_t)__builtin_amdgcn_alignbyte(q2, q1, sh) << 32);
  }
};

__device__ __forceinline__ bool narrow_ok(uint64_t a0, uint64_t a1, int32_t num_values) {
  return a1 - a0 < NARROW_LEN && (uint32_t)num_values < NARROW_VALUES;
}

__device__ __forceinline__ GSrc32 gsrc32(const uint8_t* base, uint64_t a0, uint64_t a1) {
  GSrc32 s;
  const uintptr_t b = (uintptr_t)(base + a0);
  s.abase = (glb_u32*)(b & ~(uintptr_t)3);
  s.m = (uint32_t)(b & 3);
  s.len = a1 > a0 ? (uint32_t)(a1 - a0) : 0u;
  return s;
}

// ---------------------------------------------------------------------------
// wave and workgroup scans
// ---------------------------------------------------------------------------
// Inclusive wave scans with DPP moves (no LDS): row_shr 1, 2, 4, 8 scan each
// row of 16 lanes, then row_bcast:15 and row_bcast:31 carry the rows' totals
// into rows 1, 3 and 2, 3.  Lanes whose source is outside the row read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp0(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
constexpr int DPP_ROW_SHR = 0x110, DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += dpp0<DPP_ROW_SHR | 1, 0xf>(v);
  v += dpp0<DPP_ROW_SHR | 2, 0xf>(v);
  v += dpp0<DPP_ROW_SHR | 4, 0xf>(v);
  v += dpp0<DPP_ROW_SHR | 8, 0xf>(v);
  v += dpp0<DPP_BCAST15, 0xa>(v);
  v += dpp0<DPP_BCAST31, 0xc>(v);
  return v;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_add_u64(uint64_t v) {
  const uint32_t lo = dpp0<CTRL, ROWS>((uint32_t)v), hi = dpp0<CTRL, ROWS>((uint32_t)(v >> 32));
  return v + ((uint64_t)hi << 32 | lo);
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  v = dpp_add_u64<DPP_ROW_SHR | 1, 0xf>(v);
  v = dpp_add_u64<DPP_ROW_SHR | 2, 0xf>(v);
  v = dpp_add_u64<DPP_ROW_SHR | 4, 0xf>(v);
  v = dpp_add_u64<DPP_ROW_SHR | 8, 0xf>(v);
  v = dpp_add_u64<DPP_BCAST15, 0xa>(v);
  v = dpp_add_u64<DPP_BCAST31, 0xc>(v);
  return v;
}

__device__ __forceinline__ uint64_t wave_read_u64(uint64_t v, int lane) {
  return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane) |
         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane) << 32);
}

// Orders this wave's LDS accesses (no other wave takes part).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// bits of `m` below this lane
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ---------------------------------------------------------------------------
// the tile of a wave
// ---------------------------------------------------------------------------
struct WaveTile {
  ColScan cs;
  TileDev td;
  PageDev pg;
  Streams st;
  uint32_t t;      // file-wide tile index
  uint32_t nrows;
  int64_t out0;    // output row of the tile's first row
};

// The segment holding `unit` (the last one whose first unit is at most
// `unit`): a scan of the inline table, or a binary search of the device
// table of a launch with more than MAX_SEGS segments.
__device__ __forceinline__ Segment seg_lookup(const SegTable& seg, uint32_t unit) {
  if (seg.n <= MAX_SEGS) {
    int k = 0;
    for (int j = 1; j < seg.n; ++j)
      if (seg.s[j].wg0 <= unit) k = j;
    return seg.s[k];
  }
  uint32_t lo = 0, hi = (uint32_t)seg.n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (seg.ptr[mid].wg0 <= unit) lo = mid; else hi = mid;
  }
  return seg.ptr[lo];
}

// A condition the caller knows to be the same in every lane, as the compiler
// sees it too: an early exit on it is a uniform branch (a divergent one
// would, inside the persistent kernel's tile loop, make every value that
// lives across the loop a vector register).
__device__ __forceinline__ bool uniform_bool(bool v) { return __builtin_amdgcn_readfirstlane((int)v) != 0; }

// This lane's thread index.  With LOOP (the tile functions inside the
// persistent kernel's tile loop) it is recomputed where it is used: the
// compiler would otherwise compute every per-lane constant of the tile
// functions (LDS addresses, row numbers) once, before the loop, and hold
// them all in vector registers for its whole length (twice the registers of
// the one-tile kernels).  The one-tile kernels keep the plain index, which
// the compiler may schedule freely.
template <bool LOOP>
__device__ __forceinline__ uint32_t lane_id() {
  uint32_t v = threadIdx.x;
  if constexpr (LOOP) asm volatile("" : "+v"(v));
  return v;
}

// Tile t of column table entry cs.
__device__ __forceinline__ void load_tile(const ColScan* cols, uint32_t cs, uint32_t t, uint8_t* ws, WaveTile& c) {
  c.t = t;
  c.cs = sload(cols + cs);
  c.td = sload(c.cs.fd.tiles + t);
  c.pg = sload(c.cs.fd.pages + c.td.page);
  c.nrows = (uint32_t)min((int64_t)TR, (int64_t)c.pg.num_values - c.td.row0);
  c.out0 = c.pg.row0 + c.td.row0 - c.cs.row_base;
  c.st = page_streams(c.pg, c.cs, ws);
}

// Unit (tile) of this wave: unit b * NWAVES + w of the launch, mapped to
// (column, tile) through the segment table.  False past the last unit.
__device__ __forceinline__ bool wave_tile(const SegTable& seg, const ColScan* cols, uint8_t* ws, WaveTile& c) {
  const uint32_t unit = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * NWAVES + (threadIdx.x >> 6)));
  Segment sg;
  uint32_t t;
  if (seg.spread) {
    sg = seg.s[unit % (uint32_t)seg.n];
    t = sg.t0 + unit / (uint32_t)seg.n;
  } else {
    sg = seg_lookup(seg, unit);
    t = sg.t0 + (unit - sg.wg0);
  }
  if (t >= sg.t1) return false;
  load_tile(cols, sg.cs, t, ws, c);
  return true;
}

// validity of the 64 rows of group g (word 2g: rows 64g .. 64g+31)
__device__ __forceinline__ uint64_t group_mask(uint32_t vw, uint32_t g) {
  return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)vw, (int)(2 * g)) |
         ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)vw, (int)(2 * g + 1)) << 32);
}

// ---------------------------------------------------------------------------
// RLE / bit-packed hybrid runs, decoded per lane
// ---------------------------------------------------------------------------
template <class P>
struct Hdr {
  P n;     // values of the run
  P adv;   // header + payload bytes
  P pay;   // bit-packed: bit position of the payload; RLE: the repeated value
  bool bp;
  bool ok;  // header (and an RLE value) inside the stream
};

// Run header at stream byte p of a stream of w-bit values.  With 32-bit
// positions a run's value count is capped at 2^30 and a bit-packed run whose
// payload would pass the stream end advances just past it, which the walks
// treat exactly as the uncapped run.
template <class Src>
__device__ __forceinline__ Hdr<typename Src::P> read_hdr(const Src& s, typename Src::P p, uint32_t w) {
  using P = typename Src::P;
  constexpr bool narrow = sizeof(P) == 4;
  Hdr<P> H;
  H.n = 0; H.adv = 1; H.pay = 0; H.bp = false; H.ok = false;
  if (p >= s.len) return H;
  const uint64_t a = s.window(p);  // bytes p .. p+7
  uint64_t h;
  uint32_t hl;
  if (!(a & 0x80u)) {  // one-byte header (the common case)
    h = a & 0x7fu;
    hl = 1;
  } else {
    h = 0;
    hl = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const uint32_t b = (uint32_t)(a >> (8 * k)) & 0xffu;
      if (hl == 0) {
        h |= (uint64_t)(b & 0x7fu) << (7 * k);
        if (!(b & 0x80u)) hl = k + 1;
      }
    }
  }
  H.bp = h & 1;
  const uint64_t g = h >> 1;
  const uint32_t vb = (w + 7) / 8;
  H.ok = hl != 0 && (uint64_t)p + hl <= s.len;
  if (H.bp) {
    const uint64_t n = g * 8, adv = hl + g * w;
    if constexpr (narrow) {
      H.n = (P)min(n, (uint64_t)1 << 30);
      H.adv = (P)min(adv, (uint64_t)s.len - p + 1);
    } else {
      H.n = n;
      H.adv = adv;
    }
    H.pay = (p + hl) * 8;
  } else {
    H.n = narrow ? (P)min(g, (uint64_t)1 << 30) : (P)g;
    H.adv = hl + vb;
    uint64_t v = hl ? a >> (8 * hl) : 0;  // bytes hl .. 7
    if (hl + vb > 8) v |= (uint64_t)s.byte(p + 8) << (8 * (8 - hl));
    H.pay = (P)(vb >= 4 ? (uint64_t)(uint32_t)v : (v & ((1ull << (8 * vb)) - 1)));
    if ((uint64_t)p + hl + vb > s.len) H.ok = false;
  }
  if (hl == 0) H.adv = 1;
  return H;
}

// Hands every piece of the values [a, b) to f(lo, hi, bp, x), walking the
// runs from the header at byte p whose first value is numbered rs (rs <= a):
// x is the bit position of value lo (bit-packed) or the repeated value (RLE).
// Values of a bit-packed run past the stream end, and level values above 1,
// make it return false.
template <class Src, class F>
__device__ __forceinline__ bool walk_runs(const Src& s, typename Src::P p, typename Src::I rs, uint32_t w, bool levels,
                                          typename Src::I a, typename Src::I b, F&& f) {
  using P = typename Src::P;
  using I = typename Src::I;
  while (rs < b) {
    const Hdr<P> H = read_hdr(s, p, w);
    if (!H.ok || (levels && !H.bp && H.pay > 1)) return false;
    const I re = rs + (I)H.n;
    if (re > a) {
      const I lo = max(a, rs), hi = min(b, re);
      if (H.bp) {
        if (((uint64_t)H.pay + (uint64_t)(hi - rs) * w + 7) / 8 > s.len) return false;
        f(lo, hi, true, (P)(H.pay + (P)(lo - rs) * w));
      } else {
        f(lo, hi, false, H.pay);
      }
    }
    p += H.adv;
    rs = re;
  }
  return true;
}

// Hands the pieces of values [a, b) of a hybrid stream to f (as walk_runs),
// entering at checkpoint k of the sub-tile whose first value is numbered cr
// (cr <= a): the run holding value cr is taken from the checkpoint itself, so
// a lane whose values lie in that run reads only their payload.  `entry` is
// the stream position the checkpoint offsets count from; without a recorded
// checkpoint the walk starts at (fb_pos, fb_rs), the tile's entry point.
template <class Src, class F>
__device__ __forceinline__ bool ck_walk(const Src& s, typename Src::P entry, Ck k, typename Src::I cr, uint32_t w,
                                        bool levels, typename Src::I a, typename Src::I b, typename Src::P fb_pos,
                                        typename Src::I fb_rs, F&& f) {
  using P = typename Src::P;
  using I = typename Src::I;
  if (k.at == CK_NONE) return walk_runs(s, fb_pos, fb_rs, w, levels, a, b, f);
  const I rend = cr + (I)(k.info & CK_LEFT);  // one past the run's last value
  const P pos = entry + k.at;
  const I hi = min(b, rend);
  P next;
  if (k.info >> 31) {
    const P bit0 = pos * 8 + ((k.info >> 28) & 7u);  // first bit of value cr
    if (hi > a) {
      if (((uint64_t)bit0 + (uint64_t)(hi - cr) * w + 7) / 8 > s.len) return false;
      f(a, hi, true, (P)(bit0 + (P)(a - cr) * w));
    }
    if (rend >= b) return true;
    next = (P)min(((uint64_t)bit0 + (uint64_t)(rend - cr) * w) >> 3, (uint64_t)s.len + 1);
  } else if (levels && (k.info & (1u << 29)) && rend >= b) {
    f(a, b, false, (P)((k.info >> 30) & 1u));
    return true;
  } else {
    const Hdr<P> H = read_hdr(s, pos, w);
    if (!H.ok || H.bp || (levels && H.pay > 1)) return false;
    if (hi > a) f(a, hi, false, H.pay);
    if (rend >= b) return true;
    next = pos + H.adv;
  }
  return walk_runs(s, next, rend, w, levels, max(a, rend), b, f);
}

// Definition levels of the tile: lane j (< 32) returns validity word j
// (rows 32 j .. 32 j + 31; all ones over the tile's rows for a REQUIRED
// column).  Lane l decodes rows [16 l, 16 l + 16): the run holding row 16 l
// comes from its level checkpoint (no header read), later runs are walked
// from the header after it.  False (wave-uniform) when the level stream is
// malformed.
__device__ __forceinline__ bool tile_levels(const WaveTile& c, uint32_t lk, uint32_t lane, uint32_t& vw) {
  if (!c.cs.optional) {
    const uint32_t j = lane;
    vw = 0;
    if (j < NWORDS && j * 32 < c.nrows) {
      const uint32_t rem = c.nrows - j * 32;
      vw = rem < 32 ? (1u << rem) - 1u : 0xffffffffu;
    }
    return true;
  }
  const int32_t a = (int32_t)lane * LPER, b = min((int32_t)c.nrows, a + LPER);
  uint32_t half = 0;  // levels of rows [a, a + 16)
  bool ok = true;
  auto levels = [&](const auto& ds) {
    using P = typename std::remove_reference_t<decltype(ds)>::P;
    using I = typename std::remove_reference_t<decltype(ds)>::I;
    auto put = [&](I lo, I hi, bool bp, P x) {
      const uint32_t n = (uint32_t)(hi - lo);
      const uint32_t m = bp ? (uint32_t)ds.bits(x, n) : (x ? (uint32_t)((1ull << n) - 1) : 0u);
      half |= m << (uint32_t)(lo - a);
    };
    if (lk == LCK_NONE)
      return walk_runs(ds, (P)c.td.def_pos, -(I)c.td.def_skip, 1, true, (I)a, (I)b, put);
    const P at = (P)c.td.def_pos + (P)(lk & 0xffffu);
    const uint32_t left = (lk >> 21) & 31u;
    const I hi = min((I)b, (I)(a + (int32_t)left));
    P next;
    if (lk & (1u << 19)) {  // bit-packed: the run ends on a byte boundary
      const uint32_t bo = (lk >> 16) & 7u;
      const P bit = at * 8 + bo;
      if (((uint64_t)bit + (uint64_t)(hi - a) + 7) / 8 > ds.len) return false;
      put((I)a, hi, true, bit);
      next = at + (P)((bo + left) >> 3);
    } else {
      put((I)a, hi, false, (P)((lk >> 20) & 1u));
      next = at;
    }
    if (hi >= (I)b) return true;
    return walk_runs(ds, next, hi, 1, true, hi, (I)b, put);
  };
  if (a < b) {
    if (narrow_ok(c.st.doff, c.st.dend, c.pg.num_values)) ok = levels(gsrc32(c.st.dbase, c.st.doff, c.st.dend));
    else ok = levels(gsrc(c.st.dbase, c.st.doff, c.st.dend));
  }
  const uint32_t lo16 = __shfl(half, (int)((2 * lane) & 63), 64);
  const uint32_t hi16 = __shfl(half, (int)((2 * lane + 1) & 63), 64);
  vw = lane < NWORDS ? (lo16 | (hi16 << 16)) : 0u;
  return !__ballot(!ok);
}

// Writes the tile's validity words (lane j holds word j) into the output
// bitmap.  Words that lie inside the tile (and the column's last word when it
// starts inside the tile) are stored; a word shared with a neighbouring tile
// is left to k_edges, which ORs the tiles' contributions: every tile records
// its bits of the words holding its first and its last row.
__device__ __forceinline__ void write_validity(const WaveTile& c, uint32_t vw, uint32_t lane, uint8_t* ws) {
  const int64_t out0 = c.out0, E = out0 + c.nrows;
  const int64_t w_first = out0 >> 5;
  const int64_t w_last = (E - 1) >> 5;
  const int64_t W = w_first + lane;  // at most 33 words: one per lane
  const int64_t b0 = W * 32 - out0;  // tile bit of the word's first bit
  const int32_t tw = b0 < 0 ? 0 : (int32_t)min(b0 >> 5, (int64_t)NWORDS - 1);
  const uint32_t lo = __shfl(vw, tw, 64);
  const uint32_t hi = __shfl(vw, min(tw + 1, NWORDS - 1), 64);
  if (W > w_last) return;
  uint32_t word;
  if (b0 >= 0) {
    const uint32_t sh = (uint32_t)(b0 & 31);
    word = sh ? ((lo >> sh) | ((tw + 1 < NWORDS ? hi : 0u) << (32 - sh))) : lo;
  } else {
    word = lo << (uint32_t)(-b0);
  }
  const int64_t lo_b = b0 < 0 ? -b0 : 0;
  const int64_t hi_b = (int64_t)c.nrows - b0 < 32 ? (int64_t)c.nrows - b0 : 32;
  const uint32_t mask = (hi_b >= 32 ? 0xffffffffu : ((1u << hi_b) - 1)) & (0xffffffffu << lo_b);
  word &= mask;
  if (W * 32 >= out0 && (W * 32 + 32 <= E || E == c.cs.rows))
    __builtin_nontemporal_store(word, &gptr(reinterpret_cast<uint32_t*>(c.cs.validity))[W]);
  __attribute__((address_space(1))) uint32_t* edge =
      gptr(reinterpret_cast<uint32_t*>(ws + c.cs.ws_edge)) + 2 * (size_t)(c.t - c.cs.tile_begin);
  if (W == w_first) edge[0] = word;
  if (W == w_last) edge[1] = word;
}

// Levels of the tile (validity word per lane, see tile_levels), written to
// the output bitmap of an OPTIONAL column.  False after recording an error.
__device__ __forceinline__ bool tile_validity(const WaveTile& c, uint32_t lck, uint32_t lane, uint32_t* err, uint8_t* ws,
                                              uint32_t& vw) {
  if (!tile_levels(c, lck, lane, vw)) {
    if (lane == 0) set_err(err, ERR_LEVELS, c.td.page);
    return false;
  }
  if (c.cs.optional && c.cs.validity) write_validity(c, vw, lane, ws);
  return true;
}

// Dictionary indices of the tile's values [16 lane, 16 lane + 16) into
// idx[pad(j)].  Returns 0, ERR_VALUES or ERR_DICT_INDEX (wave-uniform).
__device__ __forceinline__ uint32_t decode_indices(const WaveTile& c, Ck ck, uint32_t dn, uint32_t lane, lds_u32* idx) {
  const uint32_t w = c.pg.enc_w;
  const int32_t a = (int32_t)lane * LPER, b = min((int32_t)c.td.nn, a + LPER);
  bool ok = true, bad_idx = false;
  auto indices = [&](const auto& vs) {
    using P = typename std::remove_reference_t<decltype(vs)>::P;
    using I = typename std::remove_reference_t<decltype(vs)>::I;
    return ck_walk(vs, (P)c.td.val_pos, ck, (I)(lane >> 2) * SUB_ROWS, w, false, (I)a, (I)b, (P)c.td.val_pos,
                   -(I)c.td.val_skip, [&](I lo, I hi, bool bp, P x) {
      if (bp) {
        // a piece holds at most LPER values: every load first, then the
        // checks and the LDS stores.  Up to 24 bits, four values lie in the
        // 16 bytes from the dword holding the first one's bit (t < 104 and
        // t + w <= 128 below): one load per four values.  Wider: one per
        // value (positions past the piece repeat value lo's, which lies in
        // the stream).
        uint32_t id[LPER];
        if (w <= 24) {
          const uint32_t mask = (1u << w) - 1u;
#pragma unroll
          for (int g = 0; g < LPER / 4; ++g) {
            uint32_t sg = 0;
            const u32x4w Q = vs.quad(lo + (I)(4 * g) < hi ? x + (P)(4 * g) * w : x, sg);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint32_t t = sg + (uint32_t)j * w, k = t >> 5;
              const uint32_t a = k == 0 ? Q.x : k == 1 ? Q.y : k == 2 ? Q.z : Q.w;
              const uint32_t b = k == 0 ? Q.y : k == 1 ? Q.z : k == 2 ? Q.w : 0u;
              id[4 * g + j] = __builtin_amdgcn_alignbit(b, a, t & 31) & mask;
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < LPER; ++j) id[j] = (uint32_t)vs.bits(lo + (I)j < hi ? x + (P)j * w : x, w);
        }
#pragma unroll
        for (int j = 0; j < LPER; ++j) {
          if (lo + (I)j < hi) {
            uint32_t v = id[j];
            if (v >= dn) { bad_idx = true; v = 0; }
            idx[pad((uint32_t)(lo + (I)j))] = v;
          }
        }
      } else {
        uint32_t id = (uint32_t)x;
        if (id >= dn) { bad_idx = true; id = 0; }
        for (I v = lo; v < hi; ++v) idx[pad((uint32_t)v)] = id;
      }
    });
  };
  if (a < b) {
    if (narrow_ok(c.st.voff, c.st.vend, c.pg.num_values)) ok = indices(gsrc32(c.st.vbase, c.st.voff, c.st.vend));
    else ok = indices(gsrc(c.st.vbase, c.st.voff, c.st.vend));
  }
  if (__ballot(!ok)) return ERR_VALUES;
  if (__ballot(bad_idx)) return ERR_DICT_INDEX;
  return 0;
}

// ---------------------------------------------------------------------------
// DELTA_BINARY_PACKED terms, per lane
// ---------------------------------------------------------------------------
// Block header position of page block `bb` for tile c, whose first delta
// lies in block bu: the recorded checkpoint, else a walk over the blocks from
// the tile's entry block.  False on a malformed block.
template <class Src>
__device__ __forceinline__ bool delta_block_pos(const WaveTile& c, const Src& s, const Ck* ckv, uint32_t bb,
                                                uint32_t bu, bool is32, uint64_t& hp) {
  const uint32_t slot = bb - bu;
  if (slot < NSUB) {
    const uint32_t k = ckv[(size_t)c.t * NSUB + slot].at;
    if (k != CK_NONE) { hp = (uint64_t)c.td.val_pos + k; return true; }
  }
  const uint64_t B = c.pg.enc_w, M = c.pg.enc_m, per = B / M, total = c.pg.nonnull;
  const uint32_t maxw = is32 ? 32 : 64;
  uint64_t q = c.td.val_pos;
  for (uint64_t b = bu; b < bb; ++b) {
    int sft = 0;
    for (;;) {  // min delta
      if (q >= s.len || sft > 63) return false;
      const uint32_t x = s.byte((typename Src::P)q++);
      sft += 7;
      if (!(x & 0x80)) break;
    }
    const uint64_t left = total - 1 - b * B;
    const uint64_t used = left < B ? left : B;
    const uint64_t used_mb = (used + per - 1) / per;
    uint64_t body = 0;
    for (uint64_t m = 0; m < used_mb; ++m) {
      const uint32_t wm = s.byte((typename Src::P)(q + m));
      if (wm > maxw) return false;
      body += per * wm / 8;
    }
    q += M + body;
  }
  hp = q;
  return true;
}

// A DELTA block: its min delta, the bit position of its first miniblock and
// its (at most 16) miniblock widths.
struct DBlk {
  uint64_t md;
  uint64_t body;
  uint64_t W0, W1;
  bool ok;
};

template <class Src>
__device__ __forceinline__ DBlk delta_block(const WaveTile& c, const Src& s, const Ck* ckv, uint32_t bb, uint32_t bu,
                                            bool is32, uint32_t M) {
  DBlk k;
  uint64_t hp = 0;
  k.ok = delta_block_pos(c, s, ckv, bb, bu, is32, hp);
  if (hp > s.len) hp = s.len;
  // min delta (ULEB128, zigzag), then the miniblock widths
  const uint64_t h0 = s.window((typename Src::P)hp);
  const uint64_t h1 = (h0 & 0x8080808080808080ull) == 0x8080808080808080ull ? s.window((typename Src::P)(hp + 8)) : 0;
  uint64_t u = 0;
  uint32_t hl = 0;
#pragma unroll
  for (int j = 0; j < 10; ++j) {
    const uint32_t byte = j < 8 ? (uint32_t)(h0 >> (8 * j)) & 0xffu : (uint32_t)(h1 >> (8 * (j - 8))) & 0xffu;
    if (hl == 0) {
      u |= (uint64_t)(byte & 0x7fu) << (7 * j);
      if (!(byte & 0x80u)) hl = j + 1;
    }
  }
  if (hl == 0 || hp + hl + M > s.len) k.ok = false;
  k.md = (uint64_t)unzz(u);
  const uint64_t wb = min(hp + hl, (uint64_t)s.len);
  k.W0 = s.window((typename Src::P)wb);
  k.W1 = M > 8 ? s.window((typename Src::P)(wb + 8)) : 0;
  k.body = (wb + M) * 8;
  return k;
}

// Width of miniblock m (< 16) of block k and the bit position of its first
// value: the widths of the miniblocks before it summed with byte SADs.
__device__ __forceinline__ void delta_mini(const DBlk& k, uint32_t m, uint32_t per, uint32_t& w, uint64_t& off) {
  const uint64_t lo = m >= 8 ? ~0ull : ((1ull << (8 * m)) - 1);
  const uint64_t hi = m <= 8 ? 0ull : ((1ull << (8 * (m - 8))) - 1);
  const uint64_t a = k.W0 & lo, b = k.W1 & hi;
  uint32_t sum = __builtin_amdgcn_sad_u8((uint32_t)a, 0u, 0u);
  sum = __builtin_amdgcn_sad_u8((uint32_t)(a >> 32), 0u, sum);
  sum = __builtin_amdgcn_sad_u8((uint32_t)b, 0u, sum);
  sum = __builtin_amdgcn_sad_u8((uint32_t)(b >> 32), 0u, sum);
  w = (uint32_t)((m < 8 ? k.W0 >> (8 * m) : k.W1 >> (8 * (m - 8))) & 0xffu);
  off = k.body + (uint64_t)per * sum;
}

// D of the tile's values [16 lane, 16 lane + 16): the page's first value for
// value 0, else the delta that leads to the value.  Values past nn get 0.
// A lane's deltas lie in at most two miniblocks (a miniblock holds a multiple
// of 32 values), so it reads at most two block headers.  Returns false on a
// malformed block (wave-uniform after a ballot by the caller).
template <class Src>
__device__ __forceinline__ bool delta_terms_in(const WaveTile& c, const Src& s, const Ck* ckv, uint32_t lane,
                                               uint64_t* D) {
  const bool is32 = c.cs.type != T_INT64;  // INT32 values, or DELTA_LENGTH_BYTE_ARRAY lengths
  const uint32_t maxw = is32 ? 32 : 64;
  const uint32_t B = c.pg.enc_w, M = c.pg.enc_m, per = B / M;
#pragma unroll
  for (int q = 0; q < LPER; ++q) D[q] = 0;
  const uint32_t nn = c.td.nn, j0 = lane * LPER;
  if (j0 >= nn) return true;
  const uint32_t kk0 = c.td.k0 + j0;
  const uint32_t first = c.td.k0 == 0 ? 1u : c.td.k0;
  const uint32_t bu = (first - 1) / B;
  const uint32_t q0 = kk0 == 0 ? 1u : 0u;       // entry 0 of value 0 is the page's first value
  const uint32_t d0 = kk0 == 0 ? 0u : kk0 - 1;  // delta number of entry q0
  const uint32_t nq = min((uint32_t)LPER, nn - j0);
  if (kk0 == 0) D[0] = (uint64_t)c.pg.delta_first;
  if (q0 >= nq) return true;
  const uint32_t bbA = d0 / B, oA = d0 - bbA * B, mA = oA / per, iA = oA - mA * per;
  const DBlk A = delta_block(c, s, ckv, bbA, bu, is32, M);
  bool ok = A.ok;
  uint32_t wA, wB = 0;
  uint64_t offA, offB = 0, mdB = A.md;
  delta_mini(A, mA, per, wA, offA);
  const uint32_t nA = per - iA;  // deltas of miniblock mA from entry q0 on
  const bool needB = q0 + nA < nq;
  if (needB) {
    if (mA + 1 < M) {
      delta_mini(A, mA + 1, per, wB, offB);
    } else {
      const DBlk Bk = delta_block(c, s, ckv, bbA + 1, bu, is32, M);
      ok = ok && Bk.ok;
      mdB = Bk.md;
      delta_mini(Bk, 0, per, wB, offB);
    }
  }
  if (wA > maxw || wB > maxw) ok = false;
  const uint32_t usedA = min(nA, nq - q0);
  if ((offA + (uint64_t)(iA + usedA) * wA + 7) / 8 > s.len) ok = false;
  if (needB && (offB + (uint64_t)(nq - q0 - nA) * wB + 7) / 8 > s.len) ok = false;
  if (!ok) return false;
#pragma unroll
  for (int q = 0; q < LPER; ++q) {
    if ((uint32_t)q < q0 || (uint32_t)q >= nq) continue;
    const uint32_t r = q - q0;
    const bool inA = r < nA;
    const uint32_t w = inA ? wA : wB;
    const uint64_t bit = inA ? offA + (uint64_t)(iA + r) * wA : offB + (uint64_t)(r - nA) * wB;
    D[q] = (inA ? A.md : mdB) + s.bits64((typename Src::P)bit, w);
  }
  return true;
}

__device__ __forceinline__ bool delta_terms(const WaveTile& c, const Ck* ckv, uint32_t lane, uint64_t* D) {
  if (narrow_ok(c.st.voff, c.st.vend, c.pg.num_values))
    return delta_terms_in(c, gsrc32(c.st.vbase, c.st.voff, c.st.vend), ckv, lane, D);
  return delta_terms_in(c, gsrc(c.st.vbase, c.st.voff, c.st.vend), ckv, lane, D);
}

// ---------------------------------------------------------------------------
// string bytes: one lane copies one string of L bytes from byte S of a
// 4-byte aligned source base to byte D of a destination, 32 bytes per step:
// the aligned source dwords are loaded together, realigned with byte funnel
// shifts, and written as aligned dwords (single bytes at the string's ends).
// ---------------------------------------------------------------------------
template <class DU8, class DU32, bool NT>
__device__ __forceinline__ void copy_string(glb_u8* sbase, uint64_t S, DU8* dst, uint64_t D, uint32_t L) {
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
    DU32* dw = reinterpret_cast<DU32*>(dst + (d & ~3ull));
    const uint32_t end = dd + n;
#pragma unroll
    for (int m = 0; m < 10; ++m) {
      const uint32_t prev = m == 0 ? 0u : rr[m - 1 < 9 ? m - 1 : 8];
      const uint32_t curw = m < 9 ? rr[m] : 0u;
      const uint32_t word = dd ? __builtin_amdgcn_alignbyte(curw, prev, 4 - dd) : curw;
      const uint32_t b0 = 4u * m;
      if (b0 < end) {
        if ((m > 0 || dd == 0) && b0 + 4 <= end) {
          if constexpr (NT) __builtin_nontemporal_store(word, &dw[m]);
          else dw[m] = word;
        } else {
          DU8* b = reinterpret_cast<DU8*>(dw + m);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (b0 + k >= dd && b0 + k < end) b[k] = (uint8_t)(word >> (8 * k));
        }
      }
    }
  }
}

// One lane copies one string of L bytes from byte S of a 4-byte aligned
// source base into the wave's LDS buffer at byte D, 44 bytes per step: the
// source is read as at most three 16-byte pieces (one load instruction each),
// realigned with byte funnel shifts and written as aligned LDS dwords (single
// bytes at the string's two ends).  A step reads at most 15 bytes past the
// string.
__device__ __forceinline__ void copy_to_lds(glb_u8* sbase, uint64_t S, lds_u8* dst, uint32_t D, uint32_t L) {
  typedef uint32_t v4a __attribute__((ext_vector_type(4), aligned(4)));
  for (uint32_t j0 = 0; j0 < L; j0 += 44) {
    const uint32_t n = min(44u, L - j0);
    const uint64_t s = S + j0;
    const uint32_t d = D + j0;
    const uint32_t ss = (uint32_t)(s & 3);
    const uint32_t nsw = (ss + n + 3) >> 2;  // source dwords, <= 12
    const __attribute__((address_space(1))) v4a* q =
        reinterpret_cast<const __attribute__((address_space(1))) v4a*>(sbase + (s & ~3ull));
    uint32_t w[13];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v4a x = {0u, 0u, 0u, 0u};
      if ((uint32_t)(4 * c) < nsw) x = q[c];
      w[4 * c] = x.x; w[4 * c + 1] = x.y; w[4 * c + 2] = x.z; w[4 * c + 3] = x.w;
    }
    w[12] = 0u;
    uint32_t rr[12];  // string bytes [j0 + 4k, j0 + 4k + 4)
#pragma unroll
    for (int k = 0; k < 12; ++k) rr[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], ss);
    const uint32_t dd = d & 3;
    lds_u32* dw = reinterpret_cast<lds_u32*>(dst + (d & ~3u));
    const uint32_t end = dd + n;  // destination bytes [dd, end) of the words written
    // every index below is a compile-time constant (no register indexing)
#pragma unroll
    for (int m = 0; m < 12; ++m) {
      const uint32_t prev = m == 0 ? 0u : rr[m - 1];
      const uint32_t word = dd ? __builtin_amdgcn_alignbyte(rr[m], prev, 4 - dd) : rr[m];
      const uint32_t b0 = 4u * m;
      if (b0 < end) {
        if ((m > 0 || dd == 0) && b0 + 4 <= end) {
          dw[m] = word;
        } else {
          lds_u8* b = reinterpret_cast<lds_u8*>(dw + m);
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (b0 + k >= dd && b0 + k < end) b[k] = (uint8_t)(word >> (8 * k));
        }
      }
    }
  }
}

// The first step of copy_to_lds split in two, so that a string's loads can
// be issued one group ahead of its LDS writes: piece_load reads the (at most
// three) 16-byte pieces holding bytes [0, min(L, 44)) of the string at byte
// S; piece_write writes them to dst at byte D and copies the rest of a longer
// string directly.
__device__ __forceinline__ void piece_load(glb_u8* sbase, uint64_t S, uint32_t L, uint32_t* w) {
  typedef uint32_t v4a __attribute__((ext_vector_type(4), aligned(4)));
  const uint32_t n = min(44u, L);
  const uint32_t nsw = L ? ((uint32_t)(S & 3) + n + 3) >> 2 : 0u;
  const __attribute__((address_space(1))) v4a* q =
      reinterpret_cast<const __attribute__((address_space(1))) v4a*>(sbase + (S & ~3ull));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v4a x = {0u, 0u, 0u, 0u};
    if ((uint32_t)(4 * c) < nsw) x = q[c];
    w[4 * c] = x.x; w[4 * c + 1] = x.y; w[4 * c + 2] = x.z; w[4 * c + 3] = x.w;
  }
}

__device__ __forceinline__ void piece_write(const uint32_t* w, glb_u8* sbase, uint64_t S, lds_u8* dst, uint32_t D,
                                            uint32_t L) {
  const uint32_t n = min(44u, L);
  const uint32_t ss = (uint32_t)(S & 3);
  uint32_t rr[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) rr[k] = __builtin_amdgcn_alignbyte(k < 11 ? w[k + 1] : 0u, w[k], ss);
  const uint32_t dd = D & 3;
  lds_u32* dw = reinterpret_cast<lds_u32*>(dst + (D & ~3u));
  const uint32_t end = dd + n;
#pragma unroll
  for (int m = 0; m < 12; ++m) {
    const uint32_t prev = m == 0 ? 0u : rr[m - 1];
    const uint32_t word = dd ? __builtin_amdgcn_alignbyte(rr[m], prev, 4 - dd) : rr[m];
    const uint32_t b0 = 4u * m;
    if (b0 < end) {
      if ((m > 0 || dd == 0) && b0 + 4 <= end) {
        dw[m] = word;
      } else {
        lds_u8* b = reinterpret_cast<lds_u8*>(dw + m);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (b0 + k >= dd && b0 + k < end) b[k] = (uint8_t)(word >> (8 * k));
      }
    }
  }
  if (L > 44) copy_to_lds(sbase, S + 44, dst, D + 44, L - 44);
}

typedef __attribute__((address_space(1))) uint8_t gout_u8;
typedef __attribute__((address_space(1))) uint32_t gout_u32;

// Stores bytes [0, T) of a wave's LDS buffer to dst: aligned 16-byte chunks,
// one per lane, realigned from the LDS dwords with byte funnel shifts; the
// partial chunks at the two ends are written bytewise.
__device__ __forceinline__ void store_group(const lds_u32* buf, uint32_t nbufw, uint32_t T, gout_u8* dst,
                                            uint32_t lane) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  const uint32_t a = (uint32_t)((uintptr_t)dst & 15);
  gout_u8* d0 = dst - a;
  const uint32_t nch = (a + T + 15) >> 4;
  const uint32_t sh = (4 - (a & 3)) & 3;  // LDS byte (16 c - a) sits at this offset in its dword
  for (uint32_t c = lane; c < nch; c += 64) {
    const int32_t L0 = (int32_t)(16 * c) - (int32_t)a;
    const int32_t q0 = (L0 - (int32_t)sh) >> 2;
    uint32_t wv[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int32_t qi = q0 + k;
      wv[k] = (qi >= 0 && qi < (int32_t)nbufw) ? buf[qi] : 0u;
    }
    v4u o;
    o.x = __builtin_amdgcn_alignbyte(wv[1], wv[0], sh);
    o.y = __builtin_amdgcn_alignbyte(wv[2], wv[1], sh);
    o.z = __builtin_amdgcn_alignbyte(wv[3], wv[2], sh);
    o.w = __builtin_amdgcn_alignbyte(wv[4], wv[3], sh);
    if (L0 >= 0 && L0 + 16 <= (int32_t)T) {
      __builtin_nontemporal_store(o, reinterpret_cast<__attribute__((address_space(1))) v4u*>(d0 + 16 * c));
    } else {
      const uint32_t ow[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int32_t Lb = L0 + i;
        if (Lb >= 0 && Lb < (int32_t)T) d0[16 * c + i] = (uint8_t)(ow[i >> 2] >> (8 * (i & 3)));
      }
    }
  }
}


// Slot dictionaries: entry e's slot is the 64 bytes at 64 e; dword 0 holds
// the entry's length (at most SLOT_CHARS), its chars follow from byte 4,
// zero-padded to the slot's end.  slot_load reads the slot's first 48 bytes
// (the length and up to 44 chars) as three 16-byte pieces.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gout_u32x4;

__device__ __forceinline__ void slot_load(glb_u8* sbase, uint32_t pos, uint32_t* w) {
  const __attribute__((address_space(1))) u32x4* q =
      reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(sbase + pos);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const u32x4 x = q[c];
    w[4 * c] = x.x; w[4 * c + 1] = x.y; w[4 * c + 2] = x.z; w[4 * c + 3] = x.w;
  }
}

// ORs the L chars of a slot (its first 12 dwords in w, from slot_load) into a
// zeroed LDS buffer at byte D: dword m of the destination, counted from the
// aligned dword at D - dd (dd in 1..4, so the shift below is 0..3), is
// string bytes [4 m - dd, 4 m - dd + 4), i.e. slot bytes from 4 m + 4 - dd:
// the high bytes of slot dword m and the low bytes of dword m + 1, with the
// length dword read as zero.  Bytes outside the string are zero, so the
// neighbours' shared edge dwords combine by OR and no lane needs a mask.
// Needs 4 bytes of room before D and 64 after it.
__device__ __forceinline__ void slot_or(const uint32_t* w, glb_u8* sbase, uint32_t pos, uint32_t L, lds_u8* dst,
                                        uint32_t D) {
  const uint32_t dd = ((D - 1u) & 3u) + 1u;
  const uint32_t sh = (4u - dd) & 3u;
  lds_u32* dw = reinterpret_cast<lds_u32*>(dst + D - dd);
  uint32_t w3[5] = {0u, 0u, 0u, 0u, 0u};  // slot dwords 12..15 (chars 44..59), then past the slot
  if (L > 44) {
    const u32x4 x = reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(sbase + pos)[3];
    w3[0] = x.x; w3[1] = x.y; w3[2] = x.z; w3[3] = x.w;
  }
  uint32_t prev = 0u;  // slot dword 0 (the length) reads as zero
#pragma unroll
  for (int m = 0; m < 12; ++m) {
    const uint32_t cur = m < 11 ? w[m + 1] : w3[0];
    __hip_atomic_fetch_or(&dw[m], __builtin_amdgcn_alignbyte(cur, prev, sh), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
    prev = cur;
  }
  if (L > 44) {  // up to SLOT_CHARS
#pragma unroll
    for (int m = 12; m < 16; ++m) {
      const uint32_t cur = w3[m - 11];
      __hip_atomic_fetch_or(&dw[m], __builtin_amdgcn_alignbyte(cur, prev, sh), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_WORKGROUP);
      prev = cur;
    }
  }
}

// Stores bytes [b0, b1) of a 16-byte chunk one by one.
__device__ __forceinline__ void store_chunk_bytes(u32x4 v, gout_u8* dst, uint32_t b0, uint32_t b1) {
  const uint32_t ow[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if ((uint32_t)i >= b0 && (uint32_t)i < b1) dst[i] = (uint8_t)(ow[i >> 2] >> (8 * (i & 3)));
}


// ---------------------------------------------------------------------------
// k_snappy: one wave per compressed page (a 64-thread workgroup, so that the
// wave's 64 KiB output history fits beside another in a CU's LDS).
//
// The stream is a sequence of elements: literals (bytes copied from the
// stream) and copies (len bytes from `off` bytes back in the output).  Every
// element is written into an LDS ring holding the last SNAP_RING output
// bytes, whose byte j maps to the 16-byte aligned global address G0 + j (mod
// the ring); the ring is flushed to the page's scratch region as aligned
// 16-byte chunks.  Copies read their source from the ring (one LDS round
// trip, no wait on global stores); an offset past the ring reads the
// flushed output in global memory.  Tags are parsed from a 512-byte window
// of the stream held in two registers per lane (readlane, no memory
// latency), prefetched 256 bytes ahead; short literals come from the same
// window (ds_bpermute), long ones with 16-byte loads straight into the ring.
// ---------------------------------------------------------------------------
constexpr uint32_t SNAP_RING = 65536;
constexpr uint32_t SNAP_MASK = SNAP_RING - 1;
constexpr uint32_t SNAP_FLUSH = 4096;  // flush when this many bytes are pending
constexpr uint32_t SNAP_PIECE = 240;   // literal bytes taken from the window per step

// Stream staging: stream bytes [lo, lo + SNAP_IN) (offsets from the
// dword-aligned stream base, lo a multiple of 16) copied into LDS with
// coalesced 16-byte loads, refilled when the parse comes within SNAP_PIECE +
// 16 bytes of its end.  Offsets are 32-bit (a page is below 2 GiB).
constexpr uint32_t SNAP_IN = 2048;
struct SnapIn {
  glb_u32* base;  // dword holding stream byte 0 (minus m bytes)
  uint32_t lim;   // dwords at byte offsets >= lim are not loaded (stream end)
  uint32_t lo, hi;
  lds_u32* buf;
  __device__ __forceinline__ void fill(uint32_t a) {
    lo = a & ~15u;
    hi = lo + SNAP_IN;
    const uint32_t lane = threadIdx.x & 63;
    u32x4 v[SNAP_IN / 1024];
#pragma unroll
    for (int u = 0; u < (int)(SNAP_IN / 1024); ++u) {
      const uint32_t x = lo + 1024 * u + 16 * lane;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) v[u][kk] = x + 4 * kk < lim ? base[(x >> 2) + kk] : 0u;
    }
#pragma unroll
    for (int u = 0; u < (int)(SNAP_IN / 1024); ++u)
      *reinterpret_cast<__attribute__((address_space(3))) u32x4*>(buf + 256 * u + 4 * lane) = v[u];
    wave_sync();
  }
  // stage offset of stream byte a, with at least SNAP_PIECE + 16 bytes after it staged
  __device__ __forceinline__ uint32_t at(uint32_t a) {
    if (a < lo || a + SNAP_PIECE + 16 > hi) fill(a);
    return a - lo;
  }
  // staged bytes o .. o+4 (wave-uniform), low 5 bytes valid
  __device__ __forceinline__ uint64_t bytes8(uint32_t o) const {
    const uint32_t j = o >> 2;
    return ((uint64_t)buf[j + 1] << 32 | buf[j]) >> (8 * (o & 3));
  }
};

// Stores ring chunks [c0, c1) (16 bytes each) to g0 + 16 c: bytes [lo, hi) of
// the ring space are the page's; chunks holding others are stored bytewise.
__device__ __forceinline__ void snap_flush(const lds_u8* ring, uint8_t* g0, uint32_t c0, uint32_t c1, uint32_t lo,
                                           uint32_t hi) {
  typedef __attribute__((address_space(3))) const u32x4 lds_cv4;
  for (uint32_t c = c0 + (threadIdx.x & 63); c < c1; c += 64) {
    const u32x4 v = *reinterpret_cast<lds_cv4*>(ring + ((16 * c) & SNAP_MASK));
    const uint32_t b0 = 16 * c, b1 = b0 + 16;
    if (b0 >= lo && b1 <= hi) {
      *(gout_u32x4*)(g0 + b0) = v;
    } else {
      const uint32_t ow[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (b0 + i >= lo && b0 + i < hi) g0[b0 + i] = (uint8_t)(ow[i >> 2] >> (8 * (i & 3)));
    }
  }
}

// mode 0 (scans): the data pages without a block index; mode 1 (open): the
// pages without a block index, dictionary pages included.
__global__ __launch_bounds__(64) void k_snappy(const ColScan* cols, SegTable seg, uint8_t* ws, int mode,
                                               uint32_t* err) {
  __shared__ __align__(16) uint8_t s_ring[SNAP_RING];
  __shared__ __align__(16) uint32_t s_in[SNAP_IN / 4 + 4];
  const uint32_t gw = blockIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const Segment sg = seg_lookup(seg, gw);
  const uint32_t csi = sg.cs;
  const uint32_t p = sg.t0 + (gw - sg.wg0);
  if (p >= sg.t1) return;
  const ColScan cs = cols[csi];
  const PageDev pg = cs.fd.pages[p];
  uint32_t* sblk = cs.fd.sblk;
  if (pg.scratch_len == 0) return;
  // dictionaries are decompressed once, at open; pages with a block index
  // by k_snappy_blk
  if ((mode == 0 && pg.kind == PAGE_DICT) || (mode == 1 && !open_sel_ok(cs, pg)) || sblk[pg.sblk_begin] != SBLK_NONE)
    return;
  uint64_t src_off = pg.payload, src_len64 = pg.comp_size;
  if (pg.kind == PAGE_DATA_V2) { src_off += (uint64_t)pg.rep_len + (uint64_t)pg.def_len; src_len64 -= (uint64_t)pg.rep_len + (uint64_t)pg.def_len; }
  const uint8_t* src = cs.fd.file + src_off;
  uint8_t* dst = ws + cs.ws_scratch + (pg.scratch_off - cs.scratch_base);
  lds_u8* ring = (lds_u8*)&s_ring[0];
  const uint32_t total = pg.scratch_len;
  // stream byte i is byte m + i of the dword-aligned base; ring-space byte
  // s0 + o holds output byte o, at global address g0 + s0 + o
  const uint32_t m = (uint32_t)((uintptr_t)src & 3);
  const uint32_t s0 = (uint32_t)((uintptr_t)dst & 15);
  uint8_t* g0 = dst - s0;
  SnapIn in;
  in.base = (glb_u32*)(src - m);
  const uint32_t iend = m + (uint32_t)src_len64;  // stream bytes are [m, iend) from the base
  in.lim = iend;
  in.buf = (lds_u32*)&s_in[0];
  uint32_t ip = m;
  in.fill(ip);
  uint32_t op = 0, fc = 0;  // output bytes produced; ring-space chunks flushed
  bool bad = src_len64 >= 0x7fffffffull;
  {  // stream length (varint)
    uint64_t v = 0;
    int sft = 0;
    for (;;) {
      if (bad || ip >= iend || sft > 28) { bad = true; break; }
      const uint32_t b = (uint32_t)in.bytes8(in.at(ip++)) & 0xffu;
      v |= (uint64_t)(b & 0x7f) << sft;
      if (!(b & 0x80)) break;
      sft += 7;
    }
    if (!bad && v != total) bad = true;
  }
  while (!bad && ip < iend) {
    const uint32_t o = in.at(ip);
    const uint64_t x = in.bytes8(o);
    const uint32_t t = (uint32_t)x & 0xffu;
    const uint32_t R = s0 + op;  // ring-space position of the element's first byte
    if ((t & 3) == 0) {  // literal
      uint32_t l = t >> 2, hl = 1;
      if (l >= 60) {
        const uint32_t nb = l - 59;
        l = (uint32_t)(x >> 8) & (nb == 4 ? 0xffffffffu : ((1u << (8 * nb)) - 1));
        hl += nb;
      }
      const uint64_t L64 = (uint64_t)l + 1;
      if ((uint64_t)ip + hl + L64 > iend || L64 > total - op) { bad = true; break; }
      const uint32_t L = (uint32_t)L64;
      ip += hl;
      if (L <= SNAP_PIECE) {
        // from the window: lane q writes ring dword (R - d) / 4 + q, literal
        // bytes [4 q - d, 4 q - d + 4)
        const uint32_t ow = in.at(ip);
        const uint32_t d = R & 3;
        // stage byte of the dword's first byte (ow >= 3 unless the stage
        // starts at the literal; a negative byte is masked below)
        const int32_t so = (int32_t)ow + 4 * (int32_t)lane - (int32_t)d;
        const int32_t j0 = max(so, 0) >> 2;
        const uint32_t x0 = in.buf[j0], x1 = in.buf[j0 + 1];
        const uint32_t w = so < 0 ? x0 << (8 * (uint32_t)(-so)) : __builtin_amdgcn_alignbyte(x1, x0, (uint32_t)so & 3u);
        const int32_t b0 = 4 * (int32_t)lane - (int32_t)d;
        const uint32_t ra = R - d + 4 * lane;
        if (b0 >= 0 && b0 + 4 <= (int32_t)L) {
          *reinterpret_cast<lds_u32*>(ring + (ra & SNAP_MASK)) = w;
        } else if (b0 + 4 > 0 && b0 < (int32_t)L) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (b0 + i >= 0 && b0 + i < (int32_t)L) ring[(ra + i) & SNAP_MASK] = (uint8_t)(w >> (8 * i));
        }
      } else {
        // 16-byte loads straight into the ring: chunk c covers ring space
        // [Ra + 16 c, + 16); the literal's first and last chunks are written
        // bytewise (they share bytes with the neighbouring elements)
        const uint32_t Ra = R & ~15u, Rend = R + L;
        const uint32_t nch = (Rend - Ra + 15) >> 4;
        const uint32_t lo4 = ip & ~3u;
        for (uint32_t c0 = 0; c0 < nch; c0 += 256) {
          uint32_t wv[4][5];
          uint32_t sh[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t c = c0 + 64 * u + lane;
            const uint32_t sa = ip - (R - Ra) + 16 * c;  // stream byte (from the base) of the chunk's first byte
            sh[u] = sa & 3;
#pragma unroll
            for (int kk = 0; kk < 5; ++kk) {
              const uint32_t xo = (sa & ~3u) + 4 * kk;
              wv[u][kk] = (c < nch && xo >= lo4 && xo < iend) ? in.base[xo >> 2] : 0u;
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t c = c0 + 64 * u + lane;
            if (c >= nch) continue;
            u32x4 v;
            v.x = __builtin_amdgcn_alignbyte(wv[u][1], wv[u][0], sh[u]);
            v.y = __builtin_amdgcn_alignbyte(wv[u][2], wv[u][1], sh[u]);
            v.z = __builtin_amdgcn_alignbyte(wv[u][3], wv[u][2], sh[u]);
            v.w = __builtin_amdgcn_alignbyte(wv[u][4], wv[u][3], sh[u]);
            const uint32_t b0 = Ra + 16 * c;
            if (b0 >= R && b0 + 16 <= Rend) {
              *reinterpret_cast<__attribute__((address_space(3))) u32x4*>(ring + (b0 & SNAP_MASK)) = v;
            } else {
              const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
              for (int i = 0; i < 16; ++i)
                if (b0 + i >= R && b0 + i < Rend) ring[(b0 + i) & SNAP_MASK] = (uint8_t)(vw[i >> 2] >> (8 * (i & 3)));
            }
          }
          // a long literal must not overrun the unflushed part of the ring
          if (c0 + 256 < nch) {
            wave_sync();
            const uint32_t upto = (Ra >> 4) + c0 + 256;
            if (upto > fc) {
              snap_flush(ring, g0, fc, upto, s0, s0 + total);
              fc = upto;
            }
          }
        }
      }
      ip += L;
      op += L;
    } else {  // copy
      uint32_t len, off, hl;
      if ((t & 3) == 1) {
        hl = 2;
        len = 4 + ((t >> 2) & 7);
        off = ((t >> 5) << 8) | ((uint32_t)(x >> 8) & 0xffu);
      } else if ((t & 3) == 2) {
        hl = 3;
        len = (t >> 2) + 1;
        off = (uint32_t)(x >> 8) & 0xffffu;
      } else {
        hl = 5;
        len = (t >> 2) + 1;
        off = (uint32_t)(x >> 8);
      }
      if (ip + hl > iend || off == 0 || off > op || len > total - op) { bad = true; break; }
      ip += hl;
      // source byte of lane q: R - off + q, repeating with period off when
      // the copy overlaps its own output
      const uint32_t q = lane < len ? lane : 0u;
      uint32_t sidx;
      if (off >= len) sidx = R - off + q;
      else sidx = R - off + q % off;
      uint32_t b;
      if (off <= SNAP_RING) {
        b = ring[sidx & SNAP_MASK];
      } else {  // past the ring: from the flushed output
        __builtin_amdgcn_s_waitcnt(0);
        __threadfence_block();
        b = reinterpret_cast<volatile const uint8_t*>(g0)[sidx];
      }
      if (lane < len) ring[(R + lane) & SNAP_MASK] = (uint8_t)b;
      op += len;
    }
    const uint32_t full = (s0 + op) >> 4;
    if (full - fc >= SNAP_FLUSH / 16) {
      wave_sync();
      snap_flush(ring, g0, fc, full, s0, s0 + total);
      fc = full;
    }
  }
  if (!bad && op != total) bad = true;
  if (!bad) {
    wave_sync();
    snap_flush(ring, g0, fc, (s0 + op + 15) >> 4, s0, s0 + op);
  }
  if (bad && lane == 0) set_err(err, ERR_SNAPPY, p);
}

// k_snap_index (open): the Snappy block index of every compressed page, from
// a walk over its element tags alone, one wave per page with the stream
// staged in LDS (literal bytes are skipped, not read).  Entry b of a page is
// the stream offset of the element that starts output block b; the page's
// first entry is SBLK_NONE when an element straddles a block boundary, a
// copy reaches before the start of its block, or the stream is malformed:
// such a page is decompressed sequentially by k_snappy, which reports what
// is wrong.  The walk also counts each block's elements (sblk_ne), by which
// a scan orders its blocks.  (One lane per page, with a private LDS window
// each, was three times slower.)
__global__ __launch_bounds__(64) void k_snap_index(const ColScan* cols, SegTable seg) {
  __shared__ __align__(16) uint32_t s_in[SNAP_IN / 4 + 4];
  const uint32_t gw = blockIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const Segment sg = seg_lookup(seg, gw);
  const uint32_t p = sg.t0 + (gw - sg.wg0);
  if (p >= sg.t1) return;
  const ColScan cs = cols[sg.cs];
  const PageDev pg = cs.fd.pages[p];
  uint32_t* sblk = cs.fd.sblk;
  if (pg.scratch_len == 0 || !open_sel_ok(cs, pg)) return;
  uint64_t src_off = pg.payload, src_len64 = pg.comp_size;
  if (pg.kind == PAGE_DATA_V2) { src_off += (uint64_t)pg.rep_len + (uint64_t)pg.def_len; src_len64 -= (uint64_t)pg.rep_len + (uint64_t)pg.def_len; }
  const uint8_t* src = cs.fd.file + src_off;
  const uint32_t total = pg.scratch_len;
  const uint32_t m = (uint32_t)((uintptr_t)src & 3);
  SnapIn in;
  in.base = (glb_u32*)(src - m);
  const uint32_t iend = m + (uint32_t)min(src_len64, (uint64_t)0x7fffffffu);
  in.lim = iend;
  in.buf = (lds_u32*)&s_in[0];
  uint32_t ip = m;
  in.fill(ip);
  bool ok = src_len64 < 0x7fffffffull;
  {  // stream length (varint)
    uint64_t v = 0;
    int sft = 0;
    for (;;) {
      if (!ok || ip >= iend || sft > 28) { ok = false; break; }
      const uint32_t b = (uint32_t)in.bytes8(in.at(ip++)) & 0xffu;
      v |= (uint64_t)(b & 0x7f) << sft;
      if (!(b & 0x80)) break;
      sft += 7;
    }
    if (ok && v != total) ok = false;
  }
  const uint32_t first = ip - m;
  uint32_t op = 0, ne = 0;  // ne: elements of the current block
  while (ok && ip < iend) {
    const uint64_t x = in.bytes8(in.at(ip));
    const uint32_t t = (uint32_t)x & 0xffu;
    if (op && (op & (SNAP_BLOCK - 1)) == 0) {
      if (lane == 0) {
        sblk[pg.sblk_begin + op / SNAP_BLOCK] = ip - m;
        cs.fd.sblk_ne[pg.sblk_begin + op / SNAP_BLOCK - 1] = ne;
      }
      ne = 0;
    }
    uint32_t len, hl;
    if ((t & 3) == 0) {  // literal
      uint32_t l = t >> 2;
      hl = 1;
      if (l >= 60) {
        const uint32_t nb = l - 59;
        l = (uint32_t)(x >> 8) & (nb == 4 ? 0xffffffffu : ((1u << (8 * nb)) - 1));
        hl += nb;
      }
      const uint64_t L64 = (uint64_t)l + 1;
      if ((uint64_t)ip + hl + L64 > iend || L64 > total - op) { ok = false; break; }
      len = (uint32_t)L64;
      ip += hl + len;
    } else {  // copy
      uint32_t off;
      if ((t & 3) == 1) {
        hl = 2;
        len = 4 + ((t >> 2) & 7);
        off = ((t >> 5) << 8) | ((uint32_t)(x >> 8) & 0xffu);
      } else if ((t & 3) == 2) {
        hl = 3;
        len = (t >> 2) + 1;
        off = (uint32_t)(x >> 8) & 0xffffu;
      } else {
        hl = 5;
        len = (t >> 2) + 1;
        off = (uint32_t)(x >> 8);
      }
      if (ip + hl > iend || off == 0 || off > op || len > total - op) { ok = false; break; }
      if (off > op % SNAP_BLOCK) { ok = false; break; }  // reaches before its block
      ip += hl;
    }
    if (op / SNAP_BLOCK != (op + len - 1) / SNAP_BLOCK) { ok = false; break; }  // straddles a boundary
    op += len;
    ++ne;
  }
  if (op != total) ok = false;
  if (lane == 0 && ok && total) cs.fd.sblk_ne[pg.sblk_begin + (total - 1) / SNAP_BLOCK] = ne;
  if (lane == 0) sblk[pg.sblk_begin] = ok ? first : SBLK_NONE;
}

// One lane copies n <= 64 bytes src -> dst (no overlap) with one round of
// loads: five 16-byte loads from the source's dword (16-byte loads need only
// dword alignment) give the run, and destination dword j (dword-aligned)
// gets bytes [4 j - d, 4 j - d + 4) of it, realigned with byte funnel
// shifts.  The lane writes its block front to back, so the bytes before the
// run (the head of dword 0) are kept, written bytewise, while the at most 3
// bytes after the run's last dword are left for the next element to
// overwrite (a block ends on a 16-byte boundary, a page inside its scratch
// padding).  Reads at most 3 bytes before and 16 after the range.  The
// source may be this lane's own earlier output: a lane's loads see its
// earlier stores (program order), so no wait is needed.
typedef uint32_t u32x4a __attribute__((ext_vector_type(4), aligned(4)));
// lane_copy64 in two halves: the loads (into w), and the stores of the run
// from w (sh: the source's byte offset in its dword).
__device__ __forceinline__ void lane_load64(const uint8_t* src, uint32_t n, uint32_t (&w)[20]) {
  const uint32_t sh = (uint32_t)((uintptr_t)src & 3);
  const __attribute__((address_space(1))) u32x4a* q =
      (const __attribute__((address_space(1))) u32x4a*)((uintptr_t)src & ~(uintptr_t)3);
  const uint32_t nq = (sh + n + 3) >> 2;  // source dwords, <= 17
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    u32x4a x = {0u, 0u, 0u, 0u};
    if ((uint32_t)(4 * c) < nq) x = q[c];
    w[4 * c] = x.x; w[4 * c + 1] = x.y; w[4 * c + 2] = x.z; w[4 * c + 3] = x.w;
  }
}
__device__ __forceinline__ void lane_store64(uint8_t* dst, uint32_t sh, uint32_t n, const uint32_t (&w)[20]) {
  const uint32_t d = (uint32_t)((uintptr_t)dst & 3);
  // destination byte 4 j + i holds run byte 4 j + i - d = w byte 4 j + i + (sh - d)
  const int32_t e = (int32_t)sh - (int32_t)d;  // -3 .. 3
  const uint32_t fs = (uint32_t)e & 3u;
  const bool back = e < 0;  // the word's first byte is in w[j - 1]
  __attribute__((address_space(1))) uint32_t* dw =
      (__attribute__((address_space(1))) uint32_t*)((uintptr_t)dst & ~(uintptr_t)3);
  const uint32_t nd = (d + n + 3) >> 2;  // destination dwords, <= 17
#pragma unroll
  for (int j = 0; j < 17; ++j) {
    const uint32_t lo = back ? (j > 0 ? w[j - 1] : 0u) : w[j];
    const uint32_t hi = back ? w[j] : (j + 1 < 20 ? w[j + 1] : 0u);
    const uint32_t o = __builtin_amdgcn_alignbyte(hi, lo, fs);
    if (j == 0 && d) {
      uint8_t* bp = (uint8_t*)dw;
#pragma unroll
      for (int i = 1; i < 4; ++i)
        if ((uint32_t)i >= d && (uint32_t)i - d < n) bp[i] = (uint8_t)(o >> (8 * i));
    } else if ((uint32_t)j < nd) {
      dw[j] = o;
    }
  }
}
__device__ __forceinline__ void lane_copy64(uint8_t* dst, const uint8_t* src, uint32_t n) {
  uint32_t w[20];
  lane_load64(src, n, w);
  lane_store64(dst, (uint32_t)((uintptr_t)src & 3), n, w);
}

// The wave's active lanes (rank r of nact) copy n bytes s -> d together (a
// literal: no overlap), 16 destination bytes per lane and step, the loads of
// WC_UNROLL steps issued before their stores.  Destination dword k (counted
// from d's dword) holds source bytes [4 k - sh, 4 k - sh + 4), sh = d & 3;
// every dword is stored whole except dword 0 when d is not dword-aligned
// (its bytes before d are earlier output, written bytewise), so up to 3
// bytes after d + n are overwritten, which the owning lane's next element
// writes again (a block ends on a 16-byte boundary, a page inside its
// scratch padding).  Reads at most 3 bytes before s and 7 after s + n.
constexpr int WC_UNROLL = 2;
__device__ __forceinline__ void wave_copy(uint8_t* d, const uint8_t* s, uint32_t n, uint32_t r, uint32_t nact) {
  const uint32_t sh = (uint32_t)((uintptr_t)d & 3);
  __attribute__((address_space(1))) uint32_t* dw =
      (__attribute__((address_space(1))) uint32_t*)((uintptr_t)d & ~(uintptr_t)3);
  const uint32_t nd = (sh + n + 3) >> 2;       // destination dwords
  const uintptr_t a0 = (uintptr_t)s - sh;      // source byte of destination dword 0's first byte
  const uint32_t e = (uint32_t)(a0 & 3);
  const __attribute__((address_space(1))) uint32_t* q =
      (const __attribute__((address_space(1))) uint32_t*)(a0 & ~(uintptr_t)3);
  const uint32_t step = 4 * nact;
  for (uint32_t k0 = 4 * r; k0 < nd; k0 += WC_UNROLL * step) {
    uint32_t w[WC_UNROLL][5];
#pragma unroll
    for (int u = 0; u < WC_UNROLL; ++u) {
      const uint32_t kk = k0 + u * step;
#pragma unroll
      for (int c = 0; c < 5; ++c) w[u][c] = kk + c <= nd ? q[kk + c] : 0u;
    }
#pragma unroll
    for (int u = 0; u < WC_UNROLL; ++u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t k = k0 + u * step + j;
        const uint32_t v = __builtin_amdgcn_alignbyte(w[u][j + 1], w[u][j], e);
        if (k == 0 && sh) {
          uint8_t* bp = (uint8_t*)dw;
#pragma unroll
          for (int i = 1; i < 4; ++i)
            if ((uint32_t)i >= sh && (uint32_t)i - sh < n) bp[i] = (uint8_t)(v >> (8 * i));
        } else if (k < nd) {
          dw[k] = v;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// k_snappy_blk: the pages of the Snappy block index, one lane per 64 KiB
// output block (SNAP_LANES blocks of one or several pages advance together
// in a wave, whose other lanes join every copy of a literal longer than 64
// bytes).  A lane decodes its block in batches: up to SNAP_BATCH short
// elements (at most SNAP_SHORT bytes each) are parsed from the lane's
// SNAP_WIN-byte window of the stream in LDS, then all their sources are
// loaded (one 16-byte load each: the literal's stream bytes or the copy's
// earlier output), then all are stored, so that a batch costs one memory
// round trip instead of one per element.  A copy whose source lies in the
// batch's own output reads it from a per-lane LDS copy of that output (a
// source starting before the copy's first dword ends the batch); a longer
// element, or a copy overlapping its own output, ends the batch and is
// decoded on its own after the batch's stores (a literal of at most 64
// bytes with its stream bytes loaded beside the batch's sources).  Loads see
// the lane's earlier stores (program order), so no wait is needed between
// batches.  With sord, a scan's blocks come densest first (k_snap_order), so
// that the blocks of a wave need similar numbers of batches.
// ---------------------------------------------------------------------------
constexpr int SNAP_BATCH = 8;
constexpr uint32_t SNAP_SHORT = 13;  // a run of up to 13 bytes lies in the 16 bytes from its dword
constexpr uint32_t SNAP_WIN = 64;
constexpr uint32_t SNAP_WSTRIDE = 20;  // dwords per lane window (80 bytes: fewer bank conflicts)
// dwords per lane of the batch's output in LDS (from the dword holding the
// batch's first byte; 16 bytes per element written, at most SNAP_SHORT apart)
constexpr uint32_t SNAP_BSTRIDE = ((SNAP_BATCH * SNAP_SHORT + 20 + 15) / 16) * 4 + 4;
// One lane's block of k_snappy_blk: its page's compressed stream, output
// region and element range.  False for a lane without a block (past the
// segment, a page that is not compressed or is decoded by k_snappy).
struct SnapLane {
  const uint8_t* src;
  uint8_t* dst;
  uint32_t ip, iend, ob, oend, page, pad_;
  bool bad;
};
// Block b of column-table entry csi.
__device__ __forceinline__ bool snap_lane_at(const ColScan* cols, uint32_t csi, uint32_t b, uint8_t* ws, SnapLane& sl,
                                             bool dicts) {
  const ColScan cs = cols[csi];
  const uint32_t* sblk = cs.fd.sblk;
  const uint32_t p = cs.fd.sblk_page[b];
  const PageDev pg = cs.fd.pages[p];
  if (pg.scratch_len == 0 || (pg.kind == PAGE_DICT && !dicts)) return false;  // dictionaries: decompressed at open
  if (dicts && !open_sel_ok(cs, pg)) return false;
  const uint32_t first = pg.sblk_begin;
  if (sblk[first] == SBLK_NONE) return false;  // decoded sequentially by k_snappy
  uint64_t src_off = pg.payload, src_len64 = pg.comp_size;
  if (pg.kind == PAGE_DATA_V2) { src_off += (uint64_t)pg.rep_len + (uint64_t)pg.def_len; src_len64 -= (uint64_t)pg.rep_len + (uint64_t)pg.def_len; }
  const uint32_t total = pg.scratch_len;
  const uint32_t src_len = (uint32_t)src_len64;
  const uint32_t kb = b - first, nblk = (total + SNAP_BLOCK - 1) / SNAP_BLOCK;
  sl.src = cs.fd.file + src_off;
  sl.dst = ws + cs.ws_scratch + (pg.scratch_off - cs.scratch_base);
  sl.ip = sblk[b];
  sl.iend = kb + 1 < nblk ? sblk[b + 1] : src_len;
  sl.ob = kb * SNAP_BLOCK;  // the block's first output byte
  sl.oend = min(sl.ob + SNAP_BLOCK, total);
  sl.page = p;
  sl.bad = src_len64 >= 0x7fffffffull || sl.ip > sl.iend || sl.iend > src_len;
  return true;
}
// Lane gid's block: from the density buckets sord (when given), else from
// the segment table.
__device__ __forceinline__ bool snap_lane(const ColScan* cols, const SegTable& seg, const uint32_t* sord,
                                          uint32_t cap, uint8_t* ws, uint32_t gid, SnapLane& sl, bool dicts) {
  if (sord) {
    uint32_t base = 0, e = ~0u;
#pragma unroll
    for (uint32_t k = 0; k < SNAP_BUCKETS; ++k) {
      const uint32_t c = sord[k];
      if (gid >= base && gid - base < c) e = sord[64 + k * cap + (gid - base)];
      base += c;
    }
    if (e == ~0u) return false;
    return snap_lane_at(cols, e >> SNAP_ORD_BITS, e & ((1u << SNAP_ORD_BITS) - 1), ws, sl, dicts);
  }
  const Segment sg = seg_lookup(seg, gid);
  const uint32_t b = sg.t0 + (gid - sg.wg0);
  if (b >= sg.t1) return false;
  return snap_lane_at(cols, sg.cs, b, ws, sl, dicts);
}

// k_snap_order (scans): mode 0 clears the bucket counters sord[0 ..
// SNAP_BUCKETS); mode 1 puts every block of the segment table that
// k_snappy_blk decodes into the bucket of its element count (bucket k's list
// at sord + 64 + k cap; the order within a bucket is immaterial).
__global__ __launch_bounds__(WG) void k_snap_order(const ColScan* cols, SegTable seg, uint8_t* ws, uint32_t* sord,
                                                   uint32_t cap, int mode) {
  const uint32_t gid = blockIdx.x * WG + threadIdx.x;
  if (mode == 0) {
    if (gid < SNAP_BUCKETS) sord[gid] = 0;
    return;
  }
  const Segment sg = seg_lookup(seg, gid);
  const uint32_t b = sg.t0 + (gid - sg.wg0);
  SnapLane sl;
  const bool ok = b < sg.t1 && snap_lane_at(cols, sg.cs, b, ws, sl, false);
  uint32_t k = SNAP_BUCKETS;
  if (ok) {
    const uint32_t ne = max(cols[sg.cs].fd.sblk_ne[b], 1u);
    const uint32_t lg = 31u - (uint32_t)__builtin_clz(ne);
    k = lg >= 13u ? 0u : lg <= 6u ? SNAP_BUCKETS - 1 : 13u - lg;
  }
  // one atomic per bucket and wave; a lane's slot is its rank among the
  // wave's lanes of its bucket
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t below = (lane ? ~0ull >> (64 - lane) : 0ull);
  uint32_t slot = 0;
#pragma unroll
  for (uint32_t kb = 0; kb < SNAP_BUCKETS; ++kb) {
    const uint64_t m = __ballot(k == kb);
    if (!m) continue;
    const int lead = __builtin_ctzll(m);
    uint32_t base = 0;
    if ((int)lane == lead) base = atomicAdd(&sord[kb], (uint32_t)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readlane((int)base, lead);
    if (k == kb) slot = base + (uint32_t)__popcll(m & below);
  }
  if (ok) sord[64 + k * cap + slot] = (sg.cs << SNAP_ORD_BITS) | b;
}

// The 16 bytes from output dword k0 of a short element: bytes [sh, sh + n)
// of v (sh <= 3, n <= SNAP_SHORT) placed at byte d = dop & 3, the d bytes
// before them taken from tw (the earlier output of that dword); the bytes
// after the run are whatever v holds there.
__device__ __forceinline__ u32x4a place_short(const u32x4a v, uint32_t sh, uint32_t d, uint32_t tw) {
  // output byte 4 k + i (k = 0..3) is v byte 4 k + i + (sh - d)
  const int32_t e = (int32_t)sh - (int32_t)d;  // -3 .. 3
  const uint32_t fs = (uint32_t)e & 3u;
  const bool back = e < 0;
  const uint32_t u[6] = {0u, v.x, v.y, v.z, v.w, 0u};  // u[i + 1] = v[i]
  uint32_t o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    o[k] = __builtin_amdgcn_alignbyte(back ? u[k + 1] : u[k + 2], back ? u[k] : u[k + 1], fs);
  const uint32_t m = (1u << (8 * d)) - 1u;  // the bytes before the run
  o[0] = (o[0] & ~m) | (tw & m);
  return u32x4a{o[0], o[1], o[2], o[3]};
}

// dicts = 1 (open): dictionary pages too.  sord: the density buckets of
// k_snap_order (cap entries each), or null for the segment table's order.
__global__ __launch_bounds__(WG) void k_snappy_blk(const ColScan* cols, SegTable seg, const uint32_t* sord,
                                                   uint32_t cap, uint8_t* ws, uint32_t* err, int dicts) {
  __shared__ __align__(16) uint32_t s_win[WG / 64][SNAP_LANES][SNAP_WSTRIDE];
  __shared__ __align__(16) uint32_t s_bat[WG / 64][SNAP_LANES][SNAP_BSTRIDE];
  const uint32_t lw = threadIdx.x & 63;
  const uint32_t gid = (blockIdx.x * WG + threadIdx.x) / 64 * SNAP_LANES + lw;
  // lanes lw >= SNAP_LANES decode no block: they stay in the loop to help
  // copy long literals
  SnapLane sl = {nullptr, nullptr, 0u, 0u, 0u, 0u, 0u, 0u, false};
  const bool live = lw < SNAP_LANES && snap_lane(cols, seg, sord, cap, ws, gid, sl, dicts != 0);
  const uint8_t* src = sl.src;
  uint8_t* dst = sl.dst;
  uint32_t ip = sl.ip, op = sl.ob;
  const uint32_t iend = sl.iend, ob = sl.ob, oend = sl.oend, p = sl.page;
  bool bad = sl.bad;
  lds_u32* win = (lds_u32*)&s_win[threadIdx.x / 64][lw < SNAP_LANES ? lw : 0][0];
  lds_u32* bat = (lds_u32*)&s_bat[threadIdx.x / 64][lw < SNAP_LANES ? lw : 0][0];
  typedef const __attribute__((address_space(1))) u32x4a* gq4;
  typedef __attribute__((address_space(1))) u32x4a* gs4;
  // loads of unused batch slots and of lanes without a block read this
  // (valid, never written) address
  const uintptr_t dummy = (uintptr_t)cols;
  // the window: the SNAP_WIN stream bytes from the dword holding byte ip,
  // loaded during the previous batch (pieces that start past the stream's
  // end read the dummy address instead)
  const uintptr_t send = (uintptr_t)(src + iend);
  uintptr_t wa = 0;
  u32x4a wv[SNAP_WIN / 16];
  auto wload = [&]() {
    wa = (uintptr_t)(src + ip) & ~(uintptr_t)3;
#pragma unroll
    for (int c = 0; c < (int)(SNAP_WIN / 16); ++c) wv[c] = *(gq4)(wa + 16 * c < send ? wa + 16 * c : dummy);
  };
  wload();
  uint32_t tw = 0;  // the output dword holding byte op (its bytes before op are final)
  bool run = live && !bad && op < oend;
  while (__ballot(run)) {
    // the batch: element j is n bytes (nk[j] & 0xff; nk[j] & 0x100 marks a
    // copy, & 0x200 one whose source lies in this batch's output) to output
    // offset dop[j] from offset so[j] of the stream (a literal) or of the
    // output (a copy)
    uint32_t dop[SNAP_BATCH], so[SNAP_BATCH], nk[SNAP_BATCH];
    uint32_t nb = 0;
    // the element decoded alone after the batch: kind 1 a literal of at most
    // 64 bytes, 2 a longer literal (the whole wave copies it), 3 a copy
    // that does not overlap its output, 4 one that does
    uint32_t skind = 0, sop = 0, ssrc = 0, sn = 0, soff = 0;
    if (run) {
#pragma unroll
      for (int c = 0; c < (int)(SNAP_WIN / 16); ++c)
        *reinterpret_cast<__attribute__((address_space(3))) u32x4*>(win + 4 * c) =
            u32x4{wv[c].x, wv[c].y, wv[c].z, wv[c].w};
    }
    {
      const uint32_t bop0 = op;  // the output before bop0 is stored
      bool act = run;
#pragma unroll
      for (int j = 0; j < SNAP_BATCH; ++j) {
        // every step is computed, and applied only where `take` holds
        const uint32_t o = (uint32_t)((uintptr_t)(src + ip) - wa);
        const bool room = o + 5 <= SNAP_WIN;
        const uint32_t oc = room ? o : 0u;
        const uint32_t w0 = win[oc >> 2], w1 = win[(oc >> 2) + 1];
        const uint32_t x = __builtin_amdgcn_alignbyte(w1, w0, oc & 3);  // bytes o .. o + 3
        const uint32_t x4 = (w1 >> (8 * (oc & 3))) & 0xffu;            // byte o + 4
        const uint32_t t = x & 0xffu, ty = t & 3u, l6 = t >> 2;
        const uint32_t b1234 = (x >> 8) | (x4 << 24);  // bytes o + 1 .. o + 4
        // a literal: length l6 + 1, or (l6 >= 60) the next l6 - 59 bytes + 1
        const uint32_t nbb = l6 >= 60u ? l6 - 59u : 0u;
        const uint32_t lsh = (32u - 8u * nbb) & 31u;
        const uint32_t lext = (b1234 << lsh) >> lsh;
        const uint32_t llen = (nbb ? lext : l6) + 1u;
        // a copy with a 1-byte (ty 1), 2-byte (2) or 4-byte (3) offset
        const uint32_t c1len = 4u + (l6 & 7u), cnlen = l6 + 1u;
        const uint32_t c1off = ((t >> 5) << 8) | (b1234 & 0xffu);
        const uint32_t cnoff = b1234 & (0xffffffffu >> (ty == 2u ? 16u : 0u));
        const bool lit = ty == 0u, c1 = ty == 1u;
        const uint32_t len = lit ? llen : (c1 ? c1len : cnlen);
        const uint32_t off = c1 ? c1off : cnoff;
        const uint32_t hl = lit ? 1u + nbb : ty + 1u + (ty >> 1 & ty & 1u);
        const bool go = act & (op < oend) & room;
        const bool ipend = ip >= iend;
        const uint32_t rin = ipend ? 0u : iend - ip;  // stream bytes left
        bool bd = ipend | (hl > rin) | (len > oend - op);
        bd |= lit ? ((len == 0u) | (len > rin - hl)) : ((off == 0u) | (off > op - ob));
        bd &= go;
        const bool shortok = (len <= SNAP_SHORT) & (op + 16u <= oend) & (lit | (off >= len));
        // a source reaching into this batch's output is read from the batch's
        // copy in LDS, unless it starts before that copy's first dword
        const bool insrc = !lit & (op - off + len > bop0);
        const bool conflict = shortok & insrc & (op - off < (bop0 & ~3u));
        const bool take = go & !bd & !conflict;
        const bool bat = take & shortok;
        const bool slw = take & !shortok;
        dop[j] = op;
        so[j] = lit ? ip + hl : op - off;
        nk[j] = len | (lit ? 0u : 0x100u) | (insrc ? 0x200u : 0u);
        nb = bat ? (uint32_t)j + 1u : nb;
        const uint32_t kind = lit ? 1u + (uint32_t)(len > 64u) : 3u + (uint32_t)(off < len);
        skind = slw ? kind : skind;
        sop = slw ? op : sop;
        ssrc = slw ? ip + hl : ssrc;
        sn = slw ? len : sn;
        soff = slw ? off : soff;
        bad |= bd;
        ip = take ? ip + hl + (lit ? len : 0u) : ip;
        op = take ? op + len : op;
        act = bat;
      }
    }
    // the batch's sources, then the next window, then the batch's stores
    u32x4a v[SNAP_BATCH];
#pragma unroll
    for (int j = 0; j < SNAP_BATCH; ++j) {
      const uintptr_t a = (nk[j] & 0x100u) ? (uintptr_t)dst + so[j] : (uintptr_t)src + so[j];
      v[j] = *(gq4)(((uint32_t)j < nb && !(nk[j] & 0x200u) ? a : dummy) & ~(uintptr_t)3);
    }
    run = run && !bad;
    // a literal of at most 64 bytes decoded alone after the batch: its stream
    // bytes are loaded with the batch's sources (the stream is never written)
    uint32_t sw[20];
    if (run && skind == 1) lane_load64(src + ssrc, sn, sw);
    wload();
    // stored in order; when a later element of the batch has its source in
    // this batch's output, each element's 16 bytes also go to the batch's
    // copy in LDS (bat, from the dword holding byte bop0), where it reads them
    const uint32_t bb0 = dop[0] & ~3u;
    bool usebat = false;  // some element of the batch reads it
#pragma unroll
    for (int j = 1; j < SNAP_BATCH; ++j) usebat |= (uint32_t)j < nb && (nk[j] & 0x200u);
#pragma unroll
    for (int j = 0; j < SNAP_BATCH; ++j) {
      if ((uint32_t)j < nb) {
        const uintptr_t a = (nk[j] & 0x100u) ? (uintptr_t)dst + so[j] : (uintptr_t)src + so[j];
        const uint32_t n = nk[j] & 0xffu, d = dop[j] & 3u;
        u32x4a x = v[j];
        uint32_t sh = (uint32_t)(a & 3);
        if (nk[j] & 0x200u) {
          const uint32_t r = so[j] - bb0, k = r >> 2;
          x = u32x4a{bat[k], bat[k + 1], bat[k + 2], bat[k + 3]};
          sh = r & 3u;
        }
        const u32x4a w = place_short(x, sh, d, tw);
        *(gs4)((uintptr_t)dst + (dop[j] & ~3u)) = w;
        if (usebat) {
          const uint32_t k = ((dop[j] & ~3u) - bb0) >> 2;
          bat[k] = w.x; bat[k + 1] = w.y; bat[k + 2] = w.z; bat[k + 3] = w.w;
        }
        const uint32_t te = (d + n) >> 2;  // the dword holding the element's end
        tw = te == 0u ? w.x : te == 1u ? w.y : te == 2u ? w.z : w.w;
      }
    }
    // the element decoded alone
    bool big = false;
    if (run && skind) {
      if (skind == 1) {
        lane_store64(dst + sop, (uint32_t)((uintptr_t)(src + ssrc) & 3), sn, sw);
      } else if (skind == 2) {
        big = true;
      } else if (skind == 3) {
        lane_copy64(dst + sop, dst + sop - soff, sn);
      } else {  // bytes repeat with period soff
        uint32_t r = 0;  // k0 mod soff, carried from chunk to chunk
        for (uint32_t k0 = 0; k0 < sn; k0 += 8) {
          uint32_t bb[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            bb[j] = dst[sop - soff + r];
            r = r + 1 == soff ? 0u : r + 1;
          }
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (k0 + j < sn) dst[sop + k0 + j] = (uint8_t)bb[j];
        }
      }
    }
    // long literals, one after the other, each copied by all 64 lanes (a
    // lane's later loads see them: the wave's stores are performed in order)
    uint64_t m = __ballot(big);
    while (m) {
      const int l = __builtin_ctzll(m);
      m &= m - 1;
      const uintptr_t bd = (uintptr_t)(dst + sop), bs = (uintptr_t)(src + ssrc);
      uint8_t* d = (uint8_t*)(((uintptr_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bd >> 32), l) << 32) |
                              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bd, l));
      const uint8_t* s = (const uint8_t*)(((uintptr_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bs >> 32), l) << 32) |
                                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bs, l));
      wave_copy(d, s, (uint32_t)__builtin_amdgcn_readlane((int)sn, l), lw, 64);
    }
    // after an element decoded alone, the output dword holding op is read back
    if (run && skind && (op & 3u)) tw = *(const __attribute__((address_space(1))) uint32_t*)((uintptr_t)dst + (op & ~3u));
    run = run && op < oend;
  }
  if (!live) return;
  if (!bad && (op != oend || ip != iend)) bad = true;
  if (bad) set_err(err, ERR_SNAPPY, p);
}


// ---------------------------------------------------------------------------
// k_dba: DELTA_BYTE_ARRAY string pages, one wave per page.  Value k is the
// first prefix[k] bytes of value k - 1 followed by suffix k, a chain through
// the page, so a wave walks the page's values in order: the prefix lengths
// and the suffix lengths (two DELTA_BINARY_PACKED streams) are decoded 64 at
// a time, the previous value is kept in LDS and the suffix bytes pass
// through an LDS window.
//   mode 0 (at open): finds the page's value stream (as the index pass
//     does) and the start of its second stream and of the suffix bytes,
//     checks every prefix against the previous value's length, and stores
//     the page's facts in pages_out (x_src, x_len, x_sfx, x_chars, xlen,
//     x_total, x_scratch);
//   mode 1: writes the values in the PLAIN layout (u32 length, then the
//     bytes) into the page's expansion region, where the index pass and the
//     string kernels read them as a PLAIN page.
// At open the decompression layout and the expansion region are passed
// directly (open_scratch, open_out); in a scan they lie in the workspace.
// ---------------------------------------------------------------------------
constexpr uint32_t DBA_PREV = 16384;  // longest value (a page with a longer one: PQ_EUNSUPPORTED when scanned)
constexpr uint32_t DBA_WIN = 16384;   // suffix-byte window

// Wave-uniform byte read.
__device__ __forceinline__ uint32_t ubyte(const uint8_t* p) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)*p);
}

// A DELTA_BINARY_PACKED stream of 32-bit values read in order, every field
// wave-uniform.
struct DeltaSeq {
  const uint8_t* s;  // stream start
  uint32_t end;      // stream bytes
  uint32_t q;        // next byte after the blocks read so far
  uint32_t B, per, M, total, done, blocks;
  uint32_t last, mind;
  uint32_t mb, used_mb, in_mb, mbq, wq, w;
  bool bad, unsupported;

  __device__ uint64_t uleb() {
    uint64_t v = 0;
    for (uint32_t sh = 0;; sh += 7) {
      if (q >= end || sh > 63) { bad = true; return 0; }
      const uint32_t b = ubyte(s + q++);
      v |= (uint64_t)(b & 0x7f) << sh;
      if (!(b & 0x80)) return v;
    }
  }
  __device__ void init(const uint8_t* stream, uint32_t len) {
    s = stream; end = len; q = 0; bad = false; unsupported = false;
    const uint64_t b = uleb(), m = uleb(), t = uleb(), f = uleb();
    if (bad || b == 0 || b % 128 != 0 || m == 0 || b % m != 0 || (b / m) % 32 != 0 || t > 0x7fffffffull) { bad = true; return; }
    if (m > 16 || b > 65536) { unsupported = true; bad = true; return; }
    B = (uint32_t)b; M = (uint32_t)m; per = B / M; total = (uint32_t)t;
    last = (uint32_t)(f >> 1) ^ (0u - (uint32_t)(f & 1));  // zigzag, 32-bit
    done = 0; blocks = 0; mb = used_mb = 0; in_mb = 0; mbq = q; wq = q; w = 0;
  }
  __device__ void start_mb() {
    w = ubyte(s + wq + mb);
    if (w > 32 || (uint64_t)mbq + (uint64_t)per * w / 8 > end) bad = true;
  }
  __device__ void next_block() {
    const uint64_t md = uleb();
    mind = (uint32_t)(md >> 1) ^ (0u - (uint32_t)(md & 1));
    if (bad || M > end - q) { bad = true; return; }
    wq = q;
    q += M;
    const uint32_t left = total - 1 - blocks * B;
    const uint32_t used = left < B ? left : B;
    used_mb = (used + per - 1) / per;
    mb = 0; in_mb = 0; mbq = q;
    ++blocks;
    start_mb();
  }
  // the next n (<= 64, <= total - done) values into buf[0, n)
  __device__ void fill(__attribute__((address_space(3))) uint32_t* buf, uint32_t n, uint32_t lane) {
    uint32_t o = 0;
    if (done == 0 && n) {
      if (lane == 0) buf[0] = last;
      o = 1;
      done = 1;
    }
    while (o < n && !bad) {
      if (mb >= used_mb) { next_block(); if (bad) break; }
      const uint32_t cnt = min(n - o, per - in_mb);
      uint32_t d = 0;
      if (lane < cnt && w) {
        const uint64_t bit = (uint64_t)(in_mb + lane) * w;
        const uintptr_t a = (uintptr_t)(s + mbq + (bit >> 3));
        const __attribute__((address_space(1))) uint32_t* al = (const __attribute__((address_space(1))) uint32_t*)(a & ~(uintptr_t)3);
        const uint32_t sh = (uint32_t)(a & 3) * 8 + (uint32_t)(bit & 7);
        const uint64_t x = (((uint64_t)al[1] << 32) | al[0]) >> sh;
        d = w == 32 ? (uint32_t)x : (uint32_t)x & ((1u << w) - 1u);
      }
      const uint32_t incl = wave_incl_scan_u32(lane < cnt ? mind + d : 0u);
      const uint32_t v = last + incl;
      if (lane < cnt) buf[o + lane] = v;
      last = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)(cnt - 1));
      o += cnt; done += cnt; in_mb += cnt;
      if (in_mb == per) {
        mbq += per * w / 8;
        ++mb;
        in_mb = 0;
        if (mb < used_mb) start_mb();
        else q = mbq;
      }
    }
  }
};

__global__ __launch_bounds__(64) void k_dba(const ColScan* cols, SegTable seg, uint8_t* ws, const uint8_t* open_scratch,
                                            uint8_t* open_out, PageDev* pages_out, int mode, uint32_t* err) {
  __shared__ uint32_t s_p[64], s_s[64];
  __shared__ __align__(16) uint8_t s_prev[DBA_PREV];
  __shared__ __align__(16) uint8_t s_win[DBA_WIN + 32];
  const uint32_t lane = threadIdx.x & 63;
  const Segment sg = seg_lookup(seg, blockIdx.x);
  const uint32_t p = sg.t0 + (blockIdx.x - sg.wg0);
  if (p >= sg.t1) return;
  const ColScan* csp = cols + sg.cs;
  const FileDev fd = csp->fd;
  const PageDev pg = fd.pages[p];
  if (pg.kind == PAGE_DICT || pg.encoding != E_DBA || csp->type != T_BYTE_ARRAY) return;
  // the decompression layout (file-wide offsets)
  const uint8_t* sbase = open_scratch ? open_scratch : ws + csp->ws_scratch - csp->scratch_base;
  typedef __attribute__((address_space(3))) uint32_t lds_w32;
  lds_w32* bp = (lds_w32*)&s_p[0];
  lds_w32* bs = (lds_w32*)&s_s[0];
  if (mode == 0) {
    // the value stream, as the index pass finds it
    const bool in_scratch = pg.scratch_len > 0;
    uint64_t vo = 0, vl = 0;
    bool bad = false;
    const uint8_t* base = in_scratch ? sbase : fd.file;
    if (pg.kind == PAGE_DATA) {
      const uint64_t off = in_scratch ? pg.scratch_off : pg.payload, blen = pg.uncomp_size;
      if (csp->optional) {
        if (blen < 4) bad = true;
        else {
          const uint64_t L = ubyte(base + off) | ubyte(base + off + 1) << 8 | ubyte(base + off + 2) << 16 |
                             (uint64_t)ubyte(base + off + 3) << 24;
          if (L > blen - 4) bad = true;
          vo = off + 4 + L;
          vl = blen - 4 - L;
        }
      } else {
        vo = off;
        vl = blen;
      }
    } else if (in_scratch) {
      vo = pg.scratch_off;
      vl = pg.scratch_len;
    } else {
      const uint64_t lv = (uint64_t)pg.rep_len + (uint64_t)pg.def_len;
      vo = pg.payload + lv;
      vl = lv <= pg.comp_size ? pg.comp_size - lv : 0;
    }
    if (bad || vl >= 0x80000000ull) { if (lane == 0) set_err(err, ERR_STRING, p); return; }
    const uint8_t* src = base + vo;
    DeltaSeq P, S;
    P.init(src, (uint32_t)vl);
    // the prefix stream to its end: the suffix-length stream starts there
    while (!P.bad && P.done < P.total) P.fill(bp, min(64u, P.total - P.done), lane);
    // a stream ends after the miniblock holding its last value (padded)
    if (!P.bad && P.mb < P.used_mb) P.q = P.mbq + P.per * P.w / 8;
    const uint32_t sfx = P.q;
    if (!P.bad) S.init(src + sfx, (uint32_t)vl - sfx);
    while (!P.bad && !S.bad && S.done < S.total) S.fill(bs, min(64u, S.total - S.done), lane);
    if (!S.bad && S.mb < S.used_mb) S.q = S.mbq + S.per * S.w / 8;
    const uint32_t chars = sfx + S.q;
    if (P.unsupported || S.unsupported) {  // valid, but not decoded here: reported when scanned
      if (lane == 0) pages_out[p].x_total = DBA_UNSUPPORTED;
      return;
    }
    if (P.bad || S.bad || S.total != P.total) {
      if (lane == 0) set_err(err, ERR_DELTA, p);
      return;
    }
    // again side by side: every prefix within the previous value, every
    // value at most DBA_PREV bytes, the suffix bytes within the stream
    P.init(src, (uint32_t)vl);
    S.init(src + sfx, (uint32_t)vl - sfx);
    uint64_t prevlen = 0, sum = 0, sfx_sum = 0;
    uint32_t code = 0;
    while (P.done < P.total && !code) {
      const uint32_t n = min(64u, P.total - P.done);
      P.fill(bp, n, lane);
      S.fill(bs, n, lane);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (uint32_t j = 0; j < n; ++j) {
        const uint64_t pl = (uint32_t)__builtin_amdgcn_readfirstlane((int)bp[j]);
        const uint64_t sl = (uint32_t)__builtin_amdgcn_readfirstlane((int)bs[j]);
        if (pl > prevlen || (int32_t)pl < 0 || (int32_t)sl < 0) { code = ERR_STRING; break; }
        if (pl + sl > DBA_PREV) { code = ERR_UNSUPPORTED; break; }
        prevlen = pl + sl;
        sum += 4 + pl + sl;
        sfx_sum += sl;
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (!code && ((uint64_t)chars + sfx_sum > vl || sum >= 0x80000000ull)) code = ERR_STRING;
    if (code == ERR_UNSUPPORTED) { if (lane == 0) pages_out[p].x_total = DBA_UNSUPPORTED; return; }
    if (code) { if (lane == 0) set_err(err, code, p); return; }
    if (lane == 0) {
      PageDev& o = pages_out[p];
      o.x_src = vo;
      o.x_len = (uint32_t)vl;
      o.x_sfx = sfx;
      o.x_chars = chars;
      o.xlen = (uint32_t)sum;
      o.x_total = P.total;
      o.x_scratch = in_scratch ? 1u : 0u;
    }
    return;
  }
  // mode 1: the values in the PLAIN layout
  if (pg.x_total == DBA_UNSUPPORTED) return;
  const uint8_t* src = (pg.x_scratch ? sbase : fd.file) + pg.x_src;
  uint8_t* out = open_out ? open_out + pg.x_off : ws + csp->ws_xscratch + (pg.x_off - csp->xscratch_base);
  DeltaSeq P, S;
  P.init(src, pg.x_len);
  S.init(src + pg.x_sfx, pg.x_len - pg.x_sfx);
  if (P.bad || S.bad) { if (lane == 0) set_err(err, ERR_DELTA, p); return; }
  const uint8_t* chars = src + pg.x_chars;
  const uint32_t nchars = pg.x_len - pg.x_chars;
  lds_u8* prev = (lds_u8*)&s_prev[0];
  lds_u8* win = (lds_u8*)&s_win[0];
  uint32_t wlo = 0, whi = 0;  // window: suffix bytes [wlo, whi) at win[0..]
  uint32_t pos = 0, c = 0;
  while (P.done < P.total) {
    const uint32_t n = min(64u, P.total - P.done);
    P.fill(bp, n, lane);
    S.fill(bs, n, lane);
    if (P.bad || S.bad) { if (lane == 0) set_err(err, ERR_DELTA, p); return; }
    wave_sync();
    for (uint32_t j = 0; j < n; ++j) {
      const uint32_t pl = (uint32_t)__builtin_amdgcn_readfirstlane((int)bp[j]);
      const uint32_t sl = (uint32_t)__builtin_amdgcn_readfirstlane((int)bs[j]);
      const uint32_t L = pl + sl;
      if (L > DBA_PREV || (uint64_t)c + sl > nchars) { if (lane == 0) set_err(err, ERR_STRING, p); return; }
      if (c < wlo || c + sl > whi) {
        // refill: suffix bytes from c (16-byte chunks from the one holding it)
        const uintptr_t g0 = (uintptr_t)(chars + c) & ~(uintptr_t)15;
        const uint32_t lead = (uint32_t)((uintptr_t)(chars + c) - g0);
        typedef const __attribute__((address_space(1))) u32x4 gv4;
        wave_sync();
        // chunks past the stream's last byte are not read (a chunk holding
        // it reads at most 15 bytes past it, inside the page's padding or
        // the bytes that follow it in the file)
        const uintptr_t gend = (uintptr_t)(chars + nchars);
        for (uint32_t k = lane; 16 * k < DBA_WIN + 16; k += 64) {
          u32x4 v = {0u, 0u, 0u, 0u};
          if (g0 + 16 * k < gend) v = *(gv4*)(g0 + 16 * k);
          *reinterpret_cast<__attribute__((address_space(3))) u32x4*>(win + 16 * k) = v;
        }
        wave_sync();
        wlo = c - lead;  // window byte i holds suffix byte wlo + i (wlo may lie before the stream: never read)
        whi = wlo + DBA_WIN + 16;
      }
      for (uint32_t i = lane; i < 4 + L; i += 64) {
        uint32_t b;
        if (i < 4) {
          b = (L >> (8 * i)) & 0xffu;
        } else if (i - 4 < pl) {
          b = prev[i - 4];
        } else {
          b = win[c - wlo + (i - 4 - pl)];
          prev[i - 4] = (uint8_t)b;
        }
        out[pos + i] = (uint8_t)b;
      }
      wave_sync();
      pos += 4 + L;
      c += sl;
    }
  }
}

// ---------------------------------------------------------------------------
// k_copy: a plain streaming copy (16-byte loads and non-temporal stores,
// grid-stride, four chunks in flight per thread), the practical ceiling a
// scan's bytes are compared with; bytes past the last whole 16-byte chunk
// are copied one by one.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_copy(uint8_t* dst, const uint8_t* src, uint64_t n) {
  typedef const __attribute__((address_space(1))) u32x4 gv4;
  const uint64_t nch = n >> 4;
  const uint64_t stride = (uint64_t)gridDim.x * WG;
  uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
  for (; i + 3 * stride < nch; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = *((gv4*)src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], (gout_u32x4*)dst + i + u * stride);
  }
  for (; i < nch; i += stride) __builtin_nontemporal_store(*((gv4*)src + i), (gout_u32x4*)dst + i);
  if (blockIdx.x == 0 && threadIdx.x < (n & 15)) dst[(nch << 4) + threadIdx.x] = src[(nch << 4) + threadIdx.x];
}

// ---------------------------------------------------------------------------
// k_prep: validity words shared by two tiles are cleared before any tile
// ORs into them; REQUIRED columns with a validity buffer get all ones.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_prep(const ColScan* cols, SegTable seg) {
  const uint32_t gid = blockIdx.x * WG + threadIdx.x;  // one thread per tile
  const Segment sg = seg_lookup(seg, gid);
  const uint32_t t = sg.t0 + (gid - sg.wg0);
  if (t >= sg.t1) return;
  const ColScan cs = cols[sg.cs];
  if (!cs.validity) return;
  const TileDev td = cs.fd.tiles[t];
  const PageDev pg = cs.fd.pages[td.page];
  const uint32_t nrows = (uint32_t)min((int64_t)TILE_ROWS, (int64_t)pg.num_values - td.row0);
  const int64_t r0 = pg.row0 + td.row0 - cs.row_base;
  uint32_t* v = reinterpret_cast<uint32_t*>(cs.validity);
  if (cs.optional) return;
  // REQUIRED: every word whose first row lies in this tile is written whole
  // (ones for rows < rows, zeros past the end)
  for (int64_t W = (r0 + 31) >> 5; W * 32 < r0 + (int64_t)nrows; ++W) {
    const int64_t left = cs.rows - W * 32;
    v[W] = left >= 32 ? 0xffffffffu : ((1u << left) - 1);
  }
}

// ---------------------------------------------------------------------------
// k_edges: validity words shared by neighbouring tiles.  One thread per tile;
// the last tile touching a shared word (the word holding its first row, when
// that word starts in an earlier tile) ORs the contributions the tiles
// recorded (their bits of the words holding their first and last rows).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_edges(const uint8_t* __restrict__ ws, const ColScan* __restrict__ cols,
                                              SegTable seg) {
  const uint32_t gid = blockIdx.x * WG + threadIdx.x;  // one thread per tile
  const Segment sg = seg_lookup(seg, gid);
  const uint32_t t = sg.t0 + (gid - sg.wg0);
  if (t >= sg.t1) return;
  const ColScan cs = cols[sg.cs];
  if (!cs.validity || !cs.optional) return;
  auto span = [&](uint32_t u, int64_t& r0) {
    const TileDev td = cs.fd.tiles[u];
    const PageDev pg = cs.fd.pages[td.page];
    r0 = pg.row0 + td.row0 - cs.row_base;
    return (uint32_t)min((int64_t)TILE_ROWS, (int64_t)pg.num_values - td.row0);
  };
  int64_t r0;
  const uint32_t nrows = span(t, r0);
  const int64_t E = r0 + nrows;
  if ((r0 & 31) == 0) return;  // the word holding the first row starts in this tile, which stored it
  const int64_t W = r0 >> 5;
  if (E < (W + 1) * 32 && E != cs.rows) return;  // a later tile also ends inside that word
  const uint32_t* edge = reinterpret_cast<const uint32_t*>(ws + cs.ws_edge);
  uint32_t word = edge[2 * (t - cs.tile_begin)];
  uint32_t u = t;
  while (r0 > W * 32 && u > cs.tile_begin) {  // earlier tiles whose last rows are in the word
    --u;
    span(u, r0);
    word |= edge[2 * (u - cs.tile_begin) + 1];
  }
  reinterpret_cast<uint32_t*>(cs.validity)[W] = word;
}

// ---------------------------------------------------------------------------
// k_dict: dictionary pages -> the handle's resident dictionaries (run once,
// when the file is opened).  One wave per unit of a DictWork entry.
// Fixed-width dictionaries whose page body cannot serve as the array (a
// compressed page, or a body not aligned to the value width): 1024 PLAIN
// values per wave (16 per lane, all loads before the stores).  String
// dictionaries: DICT_CK_PER checkpoints (STR_CK entries each, positions from
// the open-time index) per wave; the wave copies their bytes into LDS with
// coalesced loads, one lane per checkpoint walks the length prefixes there,
// and for slot dictionaries the wave then writes every entry's 64-byte slot
// (length in the first dword, then the chars, zero-padded) from LDS.  A
// string region larger than the LDS buffer (never for slot dictionaries: at
// most DICT_CK_PER * STR_CK * SLOT_BYTES bytes) is walked in global memory.
// Every lane's walk must end exactly where the next checkpoint starts (the
// last checkpoint's walk may end before the body does: trailing bytes are
// ignored), so a wrong checkpoint is reported instead of yielding wrong
// dictionary strings.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(WG) void k_dict(const PageDev* __restrict__ pages, const uint32_t* __restrict__ strck,
                                             const DictSlot* __restrict__ slots, const DictWork* __restrict__ works,
                                             uint32_t nworks, uint32_t* __restrict__ err) {
  constexpr uint32_t NE = DICT_CK_PER * STR_CK;      // entries per string unit
  constexpr uint32_t RB = NE * SLOT_BYTES;           // LDS region bytes
  constexpr uint32_t RW = RB / 4 + 32;               // + slack for the realigning reads
  __shared__ __align__(16) uint32_t s_reg[NWAVES][RW];
  __shared__ uint32_t s_pos[NWAVES][NE], s_len[NWAVES][NE];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t unit = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * NWAVES + wave));
  // the last work item whose first unit is at most `unit` (wave-uniform
  // binary search)
  uint32_t lo = 0, hi = nworks;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (works[mid].unit0 <= unit) lo = mid; else hi = mid;
  }
  const DictWork wk = works[lo];
  const uint32_t u = unit - wk.unit0;
  if (u >= wk.units) return;
  const DictSlot sl = slots[wk.slot];
  const PageDev pg = pages[sl.page];
  const uint8_t* body = sl.body;
  const uint64_t boff = sl.body_off;
  const uint32_t n = sl.n;
  if (sl.type != T_BYTE_ARRAY) {
    const uint32_t e0 = u * DICT_FIXED_PER + lane;
    if (sl.type == T_INT32) {
      uint32_t v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t e = e0 + 64 * j;
        v[j] = e < n ? ld_u32(body, boff + (uint64_t)e * 4) : 0u;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t e = e0 + 64 * j;
        if (e < n) reinterpret_cast<uint32_t*>(sl.entries)[e] = v[j];
      }
    } else {
      uint64_t v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t e = e0 + 64 * j;
        v[j] = e < n ? ld_u64(body, boff + (uint64_t)e * 8) : 0ull;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t e = e0 + 64 * j;
        if (e < n) reinterpret_cast<uint64_t*>(sl.entries)[e] = v[j];
      }
    }
    return;
  }
  // strings: (pos, len) pairs relative to the body, and the entry lengths
  uint32_t* pairs = reinterpret_cast<uint32_t*>(sl.entries);
  const bool l16 = sl.flags & DICT_LENS16;
  const uint32_t nck = (n + STR_CK - 1) / STR_CK;
  const uint32_t ck0 = u * DICT_CK_PER;
  if (ck0 >= nck) return;
  const uint32_t ck1 = min(ck0 + DICT_CK_PER, nck);
  const uint32_t e0 = ck0 * STR_CK;
  const uint64_t q0 = strck[pg.strck_begin + ck0];
  const uint64_t q1 = ck1 < nck ? (uint64_t)strck[pg.strck_begin + ck1] : (uint64_t)pg.val_len;
  if (q1 < q0 || q1 > pg.val_len) {
    if (lane == 0) set_err(err, ERR_STRING, sl.page);
    return;
  }
  // where lane's walk (checkpoint ck0 + lane) must end, relative to q0
  const uint32_t my_ck = ck0 + lane;
  const bool last_ck = my_ck + 1 >= nck;
  const uint64_t my_end = my_ck < ck1 ? (last_ck ? q1 : (uint64_t)strck[pg.strck_begin + my_ck + 1]) - q0 : 0;
  const uint64_t R = q1 - q0;
  bool bad = false;
  if (R <= RB) {
    const uint64_t a0 = boff + q0;
    const uint32_t ss = (uint32_t)(a0 & 3);
    const uint32_t nw = (uint32_t)((ss + R + 3) >> 2);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(body + (a0 & ~3ull));
    lds_u32* reg = (lds_u32*)&s_reg[wave][0];
    for (uint32_t i = lane; i < nw; i += 64) reg[i] = src[i];
    wave_sync();
    auto lds_word = [&](uint32_t y) {  // LDS bytes [y, y + 4)
      return __builtin_amdgcn_alignbyte(reg[(y >> 2) + 1], reg[y >> 2], y & 3);
    };
    if (lane < ck1 - ck0) {
      uint64_t x = (uint64_t)strck[pg.strck_begin + ck0 + lane] - q0;  // region-relative
      for (uint32_t j = 0; j < STR_CK; ++j) {
        const uint32_t e = (ck0 + lane) * STR_CK + j;
        if (e >= n) break;
        if (x + 4 > R) { bad = true; break; }
        const uint32_t l = lds_word(ss + (uint32_t)x);
        x += 4;
        if ((uint64_t)l > R - x) { bad = true; break; }
        s_pos[wave][e - e0] = ss + (uint32_t)x;
        s_len[wave][e - e0] = l;
        x += l;
      }
      if (last_ck ? x > my_end : x != my_end) bad = true;
    }
    if (__ballot(bad)) {
      if (lane == 0) set_err(err, ERR_STRING, sl.page);
      return;
    }
    wave_sync();
    // pairs and lengths of the unit's entries from LDS, all lanes, coalesced
    const uint32_t ne = min(ck1 * STR_CK, n) - e0;
    for (uint32_t i = lane; i < ne; i += 64) {
      const uint32_t l = s_len[wave][i];
      const uint32_t pos = (uint32_t)(q0 + (s_pos[wave][i] - ss));
      reinterpret_cast<uint64_t*>(pairs)[e0 + i] = (uint64_t)pos | ((uint64_t)l << 32);
      if (l16) reinterpret_cast<uint16_t*>(sl.lens)[e0 + i] = (uint16_t)l;
      else reinterpret_cast<uint32_t*>(sl.lens)[e0 + i] = l;
    }
    if (!(sl.flags & DICT_SLOTS)) return;
    // slots: 16-byte chunk c of entry e per step (slot dword 0 is the
    // length, at most SLOT_CHARS; slot dword D > 0 holds chars [4 D - 4,
    // 4 D), zero past the length)
    glb_u8* sb = gptr(sl.slots);
    for (uint32_t i = lane; i < 4 * ne; i += 64) {
      const uint32_t ei = i >> 2, c = i & 3;
      const uint32_t L = s_len[wave][ei];
      const uint32_t y = s_pos[wave][ei];  // LDS byte of the entry's first char
      u32x4 o;
      uint32_t ow[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int D = 4 * (int)c + m;
        const int keep = (int)L - (4 * D - 4);  // chars in this dword
        const uint32_t x = (D > 0 && keep > 0) ? lds_word(y + 4 * (uint32_t)D - 4) : 0u;
        ow[m] = D == 0 ? L : (keep >= 4 ? x : (keep <= 0 ? 0u : (x & ((1u << (8 * keep)) - 1u))));
      }
      o.x = ow[0]; o.y = ow[1]; o.z = ow[2]; o.w = ow[3];
      __builtin_nontemporal_store(o, (gout_u32x4*)(sb + (uint64_t)(e0 + ei) * SLOT_BYTES + 16 * c));
    }
    return;
  }
  // a region larger than the LDS buffer: one lane per checkpoint in global memory
  if (lane < ck1 - ck0) {
    uint64_t q = strck[pg.strck_begin + ck0 + lane];
    for (uint32_t j = 0; j < STR_CK; ++j) {
      const uint32_t e = (ck0 + lane) * STR_CK + j;
      if (e >= n) break;
      if ((uint64_t)pg.val_len - q < 4) { bad = true; break; }
      const uint32_t l = ld_u32(body, boff + q);
      q += 4;
      if (l > (uint64_t)pg.val_len - q) { bad = true; break; }
      pairs[2 * e] = (uint32_t)q;
      pairs[2 * e + 1] = l;
      if (l16) reinterpret_cast<uint16_t*>(sl.lens)[e] = (uint16_t)l;
      else reinterpret_cast<uint32_t*>(sl.lens)[e] = l;
      q += l;
    }
    if (!bad && (last_ck ? q - q0 > my_end : q - q0 != my_end)) bad = true;
  }
  if (__ballot(bad) && lane == 0) set_err(err, ERR_STRING, sl.page);
}

// ---------------------------------------------------------------------------
// k_str_total: offsets[rows] and the chars capacity check of each string
// column of a scan (one thread per column), from the tile prefix.
// ---------------------------------------------------------------------------
__global__ void k_str_total(const ColScan* __restrict__ cols, const int32_t* __restrict__ which, int32_t n,
                            uint32_t* __restrict__ err) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const ColScan& cs = cols[which[i]];
  const uint64_t tot = cs.fd.tpfx[cs.tile_end] - cs.fd.tpfx[cs.tile_begin];
  if (cs.offsets) cs.offsets[cs.rows] = (int64_t)tot;
  if (tot > cs.chars_capacity) set_err(err, ERR_CAPACITY, (uint32_t)cs.col);
}

// ---------------------------------------------------------------------------
// k_prepass: per-tile auxiliaries (DELTA sums, string byte counts)
// ---------------------------------------------------------------------------
// mode 1: only the DELTA sums of DELTA_LENGTH_BYTE_ARRAY length streams (the
// second tile prefix, which mode 0 then reads for their carries)
__global__ __launch_bounds__(WG) void k_prepass(uint8_t* __restrict__ ws, const ColScan* __restrict__ cols,
                                                SegTable seg, int mode, uint32_t* __restrict__ err) {
  __shared__ uint32_t s_idx[NWAVES][PADN];
  WaveTile c;
  if (!wave_tile(seg, cols, ws, c)) return;
  const Ck* ckv = c.cs.fd.ckv;
  const Ck ckx = ckv[(size_t)c.t * NSUB + ((threadIdx.x & 63) >> 2)];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __attribute__((address_space(1))) uint64_t* aux =
      gptr(reinterpret_cast<uint64_t*>(ws + c.cs.ws_tile_aux)) + (c.t - c.cs.tile_begin);
  const bool is_str = c.cs.type == T_BYTE_ARRAY;
  const int enc = c.pg.encoding;
  if (is_str && enc == E_DLBA) {
    // DELTA_LENGTH_BYTE_ARRAY: the tile's length terms; mode 1 sums them, mode
    // 0 sums the lengths (the terms' prefix on top of the tile's carry)
    uint64_t D[LPER];
    bool ok = c.td.nn == 0 || delta_terms(c, ckv, lane, D);
    if (c.td.nn == 0) {
#pragma unroll
      for (int q = 0; q < LPER; ++q) D[q] = 0;
    }
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < LPER; ++q) {
      acc += D[q];
      D[q] = acc;
    }
    uint64_t tot;
    if (mode == 1) {
      tot = wave_read_u64(wave_incl_scan_u64(acc), 63);
    } else {
      const uint64_t carry = sload(c.cs.fd.tpfx2 + c.t) - sload(c.cs.fd.tpfx2 + c.pg.tile_begin);
      const uint64_t ex = wave_incl_scan_u64(acc) - acc;
      uint64_t sum = 0;
#pragma unroll
      for (int q = 0; q < LPER; ++q) {
        if (lane * LPER + q >= c.td.nn) continue;
        const uint32_t l = (uint32_t)(carry + ex + D[q]);
        if (l >> 31) ok = false;  // a negative length
        sum += l;
      }
      tot = wave_read_u64(wave_incl_scan_u64(sum), 63);
    }
    if (__ballot(!ok)) {
      if (lane == 0) set_err(err, ERR_STRING, c.td.page);
      return;
    }
    if (lane == 0) *aux = tot;
    return;
  }
  if (mode == 1) {
    if (lane == 0) *aux = 0;
    return;
  }
  if (is_str && (enc == E_PLAIN || enc == E_DBA)) {
    if (lane == 0) *aux = (uint64_t)c.td.val_skip - c.td.val_pos - 4ull * c.td.nn;
    return;
  }
  // tiles without a count, and encodings the decode kernels report as
  // unsupported when (and only when) their column is scanned
  if (c.td.nn == 0 || (!is_str && enc != E_DELTA) || (is_str && enc != E_PLAIN_DICT && enc != E_RLE_DICT)) {
    if (lane == 0) *aux = 0;
    return;
  }
  uint64_t acc = 0;
  if (!is_str) {  // DELTA tile sum
    uint64_t D[LPER];
    const bool ok = delta_terms(c, ckv, lane, D);
    if (__ballot(!ok)) {
      if (lane == 0) set_err(err, ERR_DELTA, c.td.page);
      return;
    }
#pragma unroll
    for (int q = 0; q < LPER; ++q) acc += D[q];
  } else {  // dictionary strings: sum of entry lengths over the tile's indices
    const DictSlot sl = sload(c.cs.fd.dicts + c.pg.chunk);
    if (sl.page == ~0u) {
      if (lane == 0) set_err(err, ERR_DICT_MISSING, c.td.page);
      return;
    }
    lds_u32* idx = (lds_u32*)&s_idx[wave][0];
    const uint32_t e = (uint32_t)__builtin_amdgcn_readfirstlane((int)decode_indices(c, ckx, sl.n, lane, idx));
    if (e) {
      if (lane == 0) set_err(err, e, c.td.page);
      return;
    }
    wave_sync();
    glb_u8* lens = gptr(sl.lens);
    uint32_t l[LPER];
#pragma unroll
    for (int q = 0; q < LPER; ++q) {
      const uint32_t j = lane + 64 * q;
      l[q] = j < c.td.nn ? idx[pad(j)] : 0u;
    }
    if (sl.flags & DICT_LENS16) {
#pragma unroll
      for (int q = 0; q < LPER; ++q) l[q] = reinterpret_cast<const __attribute__((address_space(1))) uint16_t*>(lens)[l[q]];
    } else {
#pragma unroll
      for (int q = 0; q < LPER; ++q) l[q] = reinterpret_cast<glb_u32*>(lens)[l[q]];
    }
#pragma unroll
    for (int q = 0; q < LPER; ++q)
      if (lane + 64 * q >= c.td.nn) l[q] = 0;
#pragma unroll
    for (int q = 0; q < LPER; ++q) acc += l[q];
  }
  const uint64_t tot = wave_read_u64(wave_incl_scan_u64(acc), 63);
  if (lane == 0) *aux = tot;
}

// ---------------------------------------------------------------------------
// k_decode_fixed: PLAIN and dictionary INT32 / INT64 / DOUBLE tiles
// ---------------------------------------------------------------------------
// One instantiation per kind of tile (FX_DICT: dictionary pages; FX_BSS:
// BYTE_STREAM_SPLIT pages, value k's byte b at stream byte b * (the page's
// non-null values) + k; else PLAIN; FX_WIDE: 8-byte values), so that each is
// compiled for its own register
// needs; a wave whose tile is of another kind leaves at once.
enum : int { FX_DICT = 1, FX_WIDE = 2, FX_BSS = 4 };
template <int KIND, bool LOOP>
__device__ __forceinline__ void tile_fixed(const WaveTile& c, uint8_t* __restrict__ ws, uint32_t* __restrict__ err,
                                           lds_u32* wl) {
  constexpr bool is_dict = KIND & FX_DICT;
  constexpr bool is_bss = KIND & FX_BSS;
  constexpr bool w4 = !(KIND & FX_WIDE);
  // checkpoint words first: their loads overlap the tile's metadata loads
  const uint32_t lck = c.cs.fd.ckl[(size_t)c.t * NLCK + (lane_id<LOOP>() & 63)];
  const Ck ckx = c.cs.fd.ckv[(size_t)c.t * NSUB + ((lane_id<LOOP>() & 63) >> 2)];
  const int enc = c.pg.encoding;
  if (enc == E_DELTA) return;  // k_decode_delta
  const uint32_t lane = lane_id<LOOP>() & 63;
  const bool dict_page = enc == E_PLAIN_DICT || enc == E_RLE_DICT;
  const bool bss_page = enc == E_BSS;
  if (!dict_page && !bss_page && enc != E_PLAIN) {
    if (is_dict && lane == 0) set_err(err, ERR_UNSUPPORTED, c.td.page);  // reported once
    return;
  }
  if (dict_page != is_dict || bss_page != is_bss || (c.cs.width == 4) != w4) return;  // another instantiation's tile
  uint32_t vw;
  if (!uniform_bool(tile_validity(c, lck, lane, err, ws, vw))) return;
  lds_u32* idx = wl;
  glb_u8* ent = nullptr;
  if constexpr (is_dict) {
    const DictSlot sl = sload(c.cs.fd.dicts + c.pg.chunk);
    if (sl.page == ~0u) {
      if (lane == 0) set_err(err, ERR_DICT_MISSING, c.td.page);
      return;
    }
    const uint32_t e = (uint32_t)__builtin_amdgcn_readfirstlane((int)decode_indices(c, ckx, sl.n, lane, idx));
    if (e) {
      if (lane == 0) set_err(err, e, c.td.page);
      return;
    }
    ent = gptr(sl.entries);
    wave_sync();
  }
  const GSrc vs = gsrc(c.st.vbase, c.st.voff, c.st.vend);
  const uint32_t nrows = c.nrows;
  const int64_t out0 = c.out0;
  const uint64_t k0 = c.td.k0;
  // rows 64 i + lane: value ranks first, then every load of the tile, then
  // the stores (null rows load value 0 of the tile and store zero)
  uint32_t kk[NGROUPS];
  uint32_t vmask = 0;
  {
    uint32_t kb = 0;
#pragma unroll
    for (int i = 0; i < NGROUPS; ++i) {
      const uint64_t m = group_mask(vw, i);
      const uint32_t k = kb + rank_below(m);
      kb += (uint32_t)__popcll(m);
      const bool v = ((m >> lane) & 1) && k < c.td.nn;
      kk[i] = v ? k : 0u;
      vmask |= (v ? 1u : 0u) << i;
    }
  }
  if (c.td.nn == 0) vmask = 0;
  const bool any = c.td.nn != 0;
  // one branch per case outside the row loops, so that every load of a loop
  // is issued before the first wait
  if constexpr (w4) {
    __attribute__((address_space(1))) uint32_t* out = gptr(reinterpret_cast<uint32_t*>(c.cs.values));
    uint32_t x[NGROUPS];
    if (!any) {
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) x[i] = 0;
    } else if constexpr (is_dict) {
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) kk[i] = idx[pad(kk[i])];
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) x[i] = reinterpret_cast<glb_u32*>(ent)[kk[i]];
    } else if constexpr (is_bss) {
      const uint64_t nnp = c.pg.nonnull;
      glb_u8* b0 = vs.base + vs.origin + k0;
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) {
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) v |= (uint32_t)b0[(uint64_t)b * nnp + kk[i]] << (8 * b);
        x[i] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) x[i] = vs.u32((k0 + kk[i]) * 4);
    }
#pragma unroll
    for (int i = 0; i < NGROUPS; ++i) {
      const uint32_t r = 64 * i + lane;
      if (r < nrows) __builtin_nontemporal_store(((vmask >> i) & 1) ? x[i] : 0u, &out[out0 + r]);
    }
  } else {
    __attribute__((address_space(1))) uint64_t* out = gptr(reinterpret_cast<uint64_t*>(c.cs.values));
    uint64_t x[NGROUPS];
    if (!any) {
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) x[i] = 0;
    } else if constexpr (is_dict) {
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) kk[i] = idx[pad(kk[i])];
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) x[i] = reinterpret_cast<glb_u64*>(ent)[kk[i]];
    } else if constexpr (is_bss) {
      const uint64_t nnp = c.pg.nonnull;
      glb_u8* b0 = vs.base + vs.origin + k0;
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) {
        uint64_t v = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) v |= (uint64_t)b0[(uint64_t)b * nnp + kk[i]] << (8 * b);
        x[i] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NGROUPS; ++i) x[i] = vs.u64((k0 + kk[i]) * 8);
    }
#pragma unroll
    for (int i = 0; i < NGROUPS; ++i) {
      const uint32_t r = 64 * i + lane;
      if (r < nrows) __builtin_nontemporal_store(((vmask >> i) & 1) ? x[i] : 0ull, &out[out0 + r]);
    }
  }
}

template <int KIND>
__global__ __launch_bounds__(WG) void k_decode_fixed(uint8_t* __restrict__ ws, const ColScan* __restrict__ cols,
                                                     SegTable seg, uint32_t* __restrict__ err) {
  __shared__ uint32_t s_idx[NWAVES][(KIND & FX_DICT) ? PADN : 1];
  WaveTile c;
  if (!wave_tile(seg, cols, ws, c)) return;
  tile_fixed<KIND, false>(c, ws, err, (lds_u32*)&s_idx[threadIdx.x >> 6][0]);
}

// ---------------------------------------------------------------------------
// k_decode_delta: DELTA_BINARY_PACKED INT32 / INT64 tiles
// ---------------------------------------------------------------------------
// per wave: the values of one half of the tile's rows (at most TR / 2)
constexpr uint32_t DHALF = TR / 2;
constexpr uint32_t DELTA_LDS_WORDS = 2 * (DHALF + DHALF / 16 + 4);
template <bool LOOP>
__device__ __forceinline__ void tile_delta(const WaveTile& c, uint8_t* __restrict__ ws, uint32_t* __restrict__ err,
                                           lds_u32* wl) {
  const uint32_t lck = c.cs.fd.ckl[(size_t)c.t * NLCK + (lane_id<LOOP>() & 63)];
  if (c.pg.encoding != E_DELTA) return;  // k_decode_fixed
  const uint32_t lane = lane_id<LOOP>() & 63;
  uint32_t vw;
  if (!uniform_bool(tile_validity(c, lck, lane, err, ws, vw))) return;
  __attribute__((address_space(3))) uint64_t* vals = (__attribute__((address_space(3))) uint64_t*)wl;
  const uint32_t nn = c.td.nn;
  // lane l holds values 16 l .. 16 l + 15 (prefix sums, in registers)
  uint64_t V[LPER];
#pragma unroll
  for (int q = 0; q < LPER; ++q) V[q] = 0;
  if (nn > 0) {
    const bool ok = delta_terms(c, c.cs.fd.ckv, lane, V);
    if (__ballot(!ok)) {
      if (lane == 0) set_err(err, ERR_DELTA, c.td.page);
      return;
    }
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < LPER; ++q) {
      acc += V[q];
      V[q] = acc;
    }
    const uint64_t ex = wave_incl_scan_u64(acc) - acc;
    const uint64_t carry = sload(c.cs.fd.tpfx + c.t) - sload(c.cs.fd.tpfx + c.pg.tile_begin);
#pragma unroll
    for (int q = 0; q < LPER; ++q) V[q] += carry + ex;
  }
  const uint32_t nrows = c.nrows;
  const int64_t out0 = c.out0;
  // rows [0, TR/2) use values [0, cntA), rows [TR/2, TR) the rest: each half
  // goes through the LDS buffer in turn
  uint32_t cntA = 0;
#pragma unroll
  for (int i = 0; i < NGROUPS / 2; ++i) cntA += (uint32_t)__popcll(group_mask(vw, i));
  uint32_t kb = 0;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const uint32_t lo = half ? cntA : 0u, hi = half ? nn : min(cntA, nn);
    if (half) wave_sync();  // the first half's reads are done
#pragma unroll
    for (int q = 0; q < LPER; ++q) {
      const uint32_t j = lane * LPER + q;
      if (j >= lo && j < hi) vals[pad(j - lo)] = V[q];
    }
    wave_sync();
    uint64_t x[NGROUPS / 2];
#pragma unroll
    for (int ii = 0; ii < NGROUPS / 2; ++ii) {
      const int i = half * (NGROUPS / 2) + ii;
      const uint64_t m = group_mask(vw, i);
      const uint32_t k = kb + rank_below(m);
      kb += (uint32_t)__popcll(m);
      x[ii] = (((m >> lane) & 1) && k < hi) ? vals[pad(k - lo)] : 0ull;
    }
    if (c.cs.width == 4) {
      __attribute__((address_space(1))) uint32_t* out = gptr(reinterpret_cast<uint32_t*>(c.cs.values));
#pragma unroll
      for (int ii = 0; ii < NGROUPS / 2; ++ii) {
        const uint32_t r = 64 * (half * (NGROUPS / 2) + ii) + lane;
        if (r < nrows) __builtin_nontemporal_store((uint32_t)x[ii], &out[out0 + r]);
      }
    } else {
      __attribute__((address_space(1))) uint64_t* out = gptr(reinterpret_cast<uint64_t*>(c.cs.values));
#pragma unroll
      for (int ii = 0; ii < NGROUPS / 2; ++ii) {
        const uint32_t r = 64 * (half * (NGROUPS / 2) + ii) + lane;
        if (r < nrows) __builtin_nontemporal_store(x[ii], &out[out0 + r]);
      }
    }
  }
}

__global__ __launch_bounds__(WG) void k_decode_delta(uint8_t* __restrict__ ws, const ColScan* __restrict__ cols,
                                                     SegTable seg, uint32_t* __restrict__ err) {
  __shared__ uint64_t s_vals[NWAVES][DELTA_LDS_WORDS / 2];
  WaveTile c;
  if (!wave_tile(seg, cols, ws, c)) return;
  tile_delta<false>(c, ws, err, (lds_u32*)&s_vals[threadIdx.x >> 6][0]);
}

// ---------------------------------------------------------------------------
// k_decode_str: BYTE_ARRAY tiles -> offsets and chars.  The tile's rows are
// taken 64 at a time; the strings of a group are gathered into the wave's
// LDS buffer at their output offsets and stored as aligned 16-byte chunks.
// ---------------------------------------------------------------------------
// LDS words per wave of the string tiles: the value positions (indices) of
// the tile, then, once every row's (position, length) is in registers, the
// chars staging buffer.  Slot strings are staged in the index area and as
// much again (about 8.7 KB per wave: a full buffer is stored about every 300
// rows, and four workgroups still fit a CU's LDS).
template <bool SLOTS>
struct StrLds {
  static constexpr uint32_t BUFW = SLOTS ? 2 * PADN + 8 : PADN + GROUP_CHARS / 4 + 8;
};
template <bool SLOTS, bool LOOP>
__device__ __forceinline__ void tile_str(const WaveTile& c, uint8_t* __restrict__ ws, uint32_t* __restrict__ err,
                                         lds_u32* wl) {
  constexpr uint32_t BUFW = StrLds<SLOTS>::BUFW;
  constexpr uint32_t CB = (BUFW - 8) * 4;  // staged chars per batch
  // checkpoint words first: their loads overlap the tile's metadata loads
  const uint32_t lck = c.cs.fd.ckl[(size_t)c.t * NLCK + (lane_id<LOOP>() & 63)];
  const Ck ckx = c.cs.fd.ckv[(size_t)c.t * NSUB + ((lane_id<LOOP>() & 63) >> 2)];
  const uint32_t lane = lane_id<LOOP>() & 63;
  const int enc = c.pg.encoding;
  const bool is_plain = !SLOTS && (enc == E_PLAIN || enc == E_DBA);  // DELTA_BYTE_ARRAY: expanded to PLAIN
  const bool is_dlba = !SLOTS && enc == E_DLBA;
  const bool is_dict = enc == E_PLAIN_DICT || enc == E_RLE_DICT;
  DictSlot sl;
  bool slot_tile = false;
  if (is_dict) {
    sl = sload(c.cs.fd.dicts + c.pg.chunk);
    slot_tile = sl.page != ~0u && (sl.flags & DICT_SLOTS);
  }
  if (slot_tile != SLOTS) return;  // the other instantiation decodes this tile
  if (!is_plain && !is_dict && !is_dlba) {
    if (lane == 0) set_err(err, ERR_UNSUPPORTED, c.td.page);
    return;
  }
  uint32_t vw;
  if (!uniform_bool(tile_validity(c, lck, lane, err, ws, vw))) return;
  lds_u32* u = wl;
  const TileDev& td = c.td;
  glb_u8* sbase;
  uint64_t soff;
  glb_u64* pairs = nullptr;
  if (is_plain) {
    // u[pad(j)]: offset (in the value stream) of the length prefix of the
    // tile's value j, j <= nn; one lane per STR_CK checkpoint
    sbase = (glb_u8*)c.st.vbase;
    soff = c.st.voff;
    const GSrc vs = gsrc(c.st.vbase, c.st.voff, c.st.vend);
    const uint64_t vlen = vs.len;
    bool bad = false;
    if (td.nn) {
      const uint32_t ck_lo = td.k0 / STR_CK, ck_hi = (td.k0 + td.nn - 1) / STR_CK;
      for (uint32_t ck = ck_lo + lane; ck <= ck_hi; ck += 64) {
        uint64_t q = c.cs.fd.strck[c.pg.strck_begin + ck];
        for (uint32_t j = 0; j < STR_CK; ++j) {
          const uint32_t k = ck * STR_CK + j;
          if (k >= td.k0 + td.nn) break;
          if (q + 4 > vlen) { bad = true; break; }
          const uint32_t l = vs.u32(q);
          if ((uint64_t)l > vlen - q - 4) { bad = true; break; }
          if (k >= td.k0) u[pad(k - td.k0)] = (uint32_t)q;
          q += 4 + (uint64_t)l;
        }
      }
    }
    if (lane == 0) u[pad(td.nn)] = td.val_skip;
    if (__ballot(bad)) {
      if (lane == 0) set_err(err, ERR_STRING, td.page);
      return;
    }
  } else if (is_dlba) {
    // u[pad(j)]: stream position of the first char of the tile's value j,
    // j <= nn.  Lengths: the page's DELTA_BINARY_PACKED length stream, whose
    // carry into this tile comes from the second tile prefix; positions: the
    // page's chars start, the string bytes of the page's earlier tiles (tile
    // prefix), then a scan of the lengths (lane l holds values 16 l ..)
    sbase = (glb_u8*)c.st.vbase;
    soff = c.st.voff;
    const uint64_t vlen = c.st.vend - c.st.voff;
    uint64_t D[LPER];
    bool ok = td.nn == 0 || delta_terms(c, c.cs.fd.ckv, lane, D);
    if (td.nn == 0) {
#pragma unroll
      for (int q = 0; q < LPER; ++q) D[q] = 0;
    }
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < LPER; ++q) {
      acc += D[q];
      D[q] = acc;
    }
    const uint64_t carry = sload(c.cs.fd.tpfx2 + c.t) - sload(c.cs.fd.tpfx2 + c.pg.tile_begin);
    const uint64_t ex = wave_incl_scan_u64(acc) - acc;
    const uint32_t j0 = lane * LPER;
    uint64_t lsum = 0;
#pragma unroll
    for (int q = 0; q < LPER; ++q) {
      const uint32_t l = j0 + q < td.nn ? (uint32_t)(carry + ex + D[q]) : 0u;
      if (l >> 31) ok = false;
      D[q] = l;
      lsum += l;
    }
    const uint64_t incl = wave_incl_scan_u64(lsum);
    const uint64_t total = wave_read_u64(incl, 63);
    const uint64_t* tp = c.cs.fd.tpfx;
    const uint64_t cbase = (uint64_t)c.pg.chars_at + (sload(tp + c.t) - sload(tp + c.pg.tile_begin));
    if (cbase + total > vlen || cbase + total >= 0xffffffffull) ok = false;
    uint64_t at = cbase + incl - lsum;
#pragma unroll
    for (int q = 0; q < LPER; ++q) {
      if (j0 + q < td.nn) u[pad(j0 + q)] = (uint32_t)at;
      at += D[q];
    }
    if (lane == 0) u[pad(td.nn)] = (uint32_t)(cbase + total);
    if (__ballot(!ok)) {
      if (lane == 0) set_err(err, ERR_STRING, td.page);
      return;
    }
  } else {
    if (sl.page == ~0u) {
      if (lane == 0) set_err(err, ERR_DICT_MISSING, td.page);
      return;
    }
    if (SLOTS) {  // entry e's length and chars in slot e
      sbase = gptr(sl.slots);
      soff = 0;
    } else {
      sbase = (glb_u8*)sl.body;
      soff = sl.body_off;
      pairs = reinterpret_cast<glb_u64*>(gptr(sl.entries));
    }
    const uint32_t e = (uint32_t)__builtin_amdgcn_readfirstlane((int)decode_indices(c, ckx, sl.n, lane, u));
    if (e) {
      if (lane == 0) set_err(err, e, td.page);
      return;
    }
  }
  wave_sync();

  const uint64_t* tpfx = c.cs.fd.tpfx;
  const uint64_t base = sload(tpfx + c.t) - sload(tpfx + c.cs.tile_begin);
  const uint64_t tend = sload(tpfx + c.t + 1) - sload(tpfx + c.cs.tile_begin);
  if (tend - base >= 0xffffffffull) {
    if (lane == 0) set_err(err, ERR_UNSUPPORTED, td.page);
    return;
  }
  const bool fits = c.cs.chars && tend <= c.cs.chars_capacity;
  gout_u8* chars = gptr(c.cs.chars);
  __attribute__((address_space(1))) int64_t* offs = gptr(c.cs.offsets);

  // ranks of row 64 g + lane for all groups (kk: value index, vmask: valid)
  uint32_t kk[NGROUPS];
  uint32_t vmask = 0;
  {
    uint32_t kb = 0;
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) {
      const uint64_t m = group_mask(vw, g);
      const uint32_t k = kb + rank_below(m);
      kb += (uint32_t)__popcll(m);
      const bool v = ((m >> lane) & 1) && k < td.nn;
      kk[g] = v ? k : 0u;
      vmask |= (v ? 1u : 0u) << g;
    }
  }
  if constexpr (SLOTS) {
    // Slot dictionaries, one group of 64 rows at a time: the group's slots
    // (length in dword 0, chars from byte 4) are loaded one group ahead; the
    // lengths give the group's offsets (a wave scan on top of the chars of
    // the groups before it; stored after the chars, so that no load waits
    // for them), and each lane ORs its string's realigned dwords
    // into a zeroed LDS buffer with no masks (slots are zero past the
    // string, so the neighbours' edge bytes combine by OR).  LDS byte j maps
    // to the 16-byte aligned global address G0 + j, so the buffer is stored
    // as aligned 16-byte chunks; when it fills, the full chunks are stored
    // and cleared and the partial last chunk moves to the front.  Only the
    // tile's first and last chunk are stored bytewise (they share bytes with
    // the neighbouring tiles).
    constexpr uint32_t HEAD = 16;                   // room for a string's dword before byte 0
    constexpr uint32_t CAP = BUFW * 4 - HEAD - 64;  // chars + the realignment slack
    static_assert(BUFW % 4 == 0 && CAP >= 64 * SLOT_CHARS + 15, "one group of slot strings fits the buffer");
    uint32_t sp[NGROUPS];  // byte offset of row 64 g + lane's slot (a null row reads entry 0's)
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) sp[g] = td.nn ? u[pad(kk[g])] * SLOT_BYTES : 0u;
    wave_sync();
    typedef __attribute__((address_space(3))) u32x4 lds_v4u;
    lds_v4u* zb = (lds_v4u*)wl;
    if (fits)
      for (uint32_t i = lane; i < BUFW / 4; i += 64) zb[i] = u32x4{0u, 0u, 0u, 0u};
    wave_sync();
    lds_u8* cb8 = (lds_u8*)wl + HEAD;
    lds_v4u* cbv = reinterpret_cast<lds_v4u*>(cb8);
    gout_u8* tile_chars = chars + base;
    uint32_t lo = (uint32_t)((uintptr_t)tile_chars & 15);  // LDS byte of tile char bstart
    uint32_t bstart = 0, bfill = 0, tb = 0;                // tb: tile chars before group g
    bool head_foreign = lo != 0;  // LDS bytes [0, lo) of chunk 0 belong to the previous tile
    // an all-null tile reads no slot (the dictionary may be empty)
    uint32_t wc[12], wn[12], ex[NGROUPS];
#pragma unroll
    for (int k = 0; k < 12; ++k) wn[k] = 0u;
    if (td.nn) slot_load(sbase, sp[0], wn);
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) {
#pragma unroll
      for (int k = 0; k < 12; ++k) wc[k] = wn[k];
      if (td.nn && g + 1 < NGROUPS) slot_load(sbase, sp[g + 1], wn);
      const uint32_t L = ((vmask >> g) & 1) ? wc[0] : 0u;
      const uint32_t incl = wave_incl_scan_u32(L);
      const uint32_t Tg = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      const uint32_t exg = tb + incl - L;
      ex[g] = exg;
      tb += Tg;
      if (!fits || Tg == 0) continue;
      if (bfill && lo + bfill + Tg > CAP) {
        // store the full chunks, clear them, move the partial one to the front
        wave_sync();
        const uint32_t end = lo + bfill, nfull = end >> 4, tail = end & 15;
        gout_u8* g0 = tile_chars + bstart - lo;
        for (uint32_t k = lane; k < nfull; k += 64) {
          const u32x4 v = cbv[k];
          if (k == 0 && head_foreign) store_chunk_bytes(v, g0, lo, 16);
          else __builtin_nontemporal_store(v, reinterpret_cast<gout_u32x4*>(g0 + 16 * k));
          cbv[k] = u32x4{0u, 0u, 0u, 0u};
        }
        wave_sync();
        if (lane == 0 && tail) {
          cbv[0] = cbv[nfull];
          cbv[nfull] = u32x4{0u, 0u, 0u, 0u};
        }
        wave_sync();
        head_foreign = false;
        bstart += bfill;
        lo = tail;
        bfill = 0;
      }
      if (L) slot_or(wc, sbase, sp[g], L, cb8, lo + (exg - bstart));
      bfill += Tg;
    }
    if (c.cs.offsets) {
#pragma unroll
      for (int g = 0; g < NGROUPS; ++g) {
        const uint32_t r = 64 * g + lane;
        if (r < c.nrows) __builtin_nontemporal_store((int64_t)(base + ex[g]), &offs[c.out0 + r]);
      }
    }
    // the slots' lengths and the tile prefix come from the same dictionary
    // entries; a difference is reported, never hidden
    if ((uint32_t)__builtin_amdgcn_readfirstlane((int)tb) != (uint32_t)(tend - base)) {
      if (lane == 0) set_err(err, ERR_STRING, td.page);
      return;
    }
    if (!fits) return;
    wave_sync();
    const uint32_t end = lo + bfill, nst = (end + 15) >> 4, tail = end & 15;
    gout_u8* g0 = tile_chars + bstart - lo;
    for (uint32_t k = lane; k < nst; k += 64) {
      const u32x4 v = cbv[k];
      const uint32_t b0 = (k == 0 && head_foreign) ? lo : 0u;
      const uint32_t b1 = (k + 1 == nst && tail) ? tail : 16u;
      if (b0 == 0 && b1 == 16) __builtin_nontemporal_store(v, reinterpret_cast<gout_u32x4*>(g0 + 16 * k));
      else store_chunk_bytes(v, g0 + 16 * k, b0, b1);
    }
    return;
  }
  // (position, length) of row 64 g + lane for all groups, one loop per
  // source kind (no branch inside, so every gather of the tile is issued
  // before the first wait)
  uint32_t pos[NGROUPS], len[NGROUPS];
  if (td.nn == 0) {
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) { pos[g] = 0; len[g] = 0; }
  } else if (is_plain || is_dlba) {
    const uint32_t hdr = is_plain ? 4u : 0u;  // PLAIN: a u32 length before each string
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) {
      const uint32_t q0 = u[pad(kk[g])], q1 = u[pad(kk[g] + 1)];
      pos[g] = q0 + hdr;
      len[g] = q1 - q0 - hdr;
    }
  } else {
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) pos[g] = u[pad(kk[g])];
    uint64_t pr[NGROUPS];
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) pr[g] = pairs[pos[g]];
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) {
      pos[g] = (uint32_t)pr[g];
      len[g] = (uint32_t)(pr[g] >> 32);
    }
  }
#pragma unroll
  for (int g = 0; g < NGROUPS; ++g)
    if (!((vmask >> g) & 1)) len[g] = 0;
  // row offsets: exclusive scan per group, groups in row order; GB[g] is
  // the tile-relative chars offset of group g
  uint32_t ex[NGROUPS], T[NGROUPS], GB[NGROUPS];
  {
    uint32_t tb = 0;
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) {
      const uint32_t incl = wave_incl_scan_u32(len[g]);
      T[g] = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      GB[g] = tb;
      ex[g] = tb + incl - len[g];
      tb += T[g];
    }
  }
  if (c.cs.offsets) {
#pragma unroll
    for (int g = 0; g < NGROUPS; ++g) {
      const uint32_t r = 64 * g + lane;
      if (r < c.nrows) __builtin_nontemporal_store((int64_t)(base + ex[g]), &offs[c.out0 + r]);
    }
  }
  if (!fits) return;
  {
    // chars: consecutive groups are gathered into the wave's LDS buffer until
    // it is full, then the batch is stored with aligned 16-byte chunks (one
    // wait for earlier stores per batch, not per group); a group larger than
    // the buffer is copied directly.  The buffer reuses the index area, whose
    // every entry was read above.
    wave_sync();
    lds_u32* cb = wl;
    lds_u8* cb8 = (lds_u8*)cb;
    uint32_t bstart = 0, bfill = 0;  // the batch holds tile chars [bstart, bstart + bfill)
    uint32_t wc[12], wn[12];          // this group's and the next group's source pieces
    piece_load(sbase, soff + pos[0], len[0], wn);
    for (int g = 0; g < NGROUPS; ++g) {
  #pragma unroll
      for (int k = 0; k < 12; ++k) wc[k] = wn[k];
      if (g + 1 < NGROUPS) piece_load(sbase, soff + pos[g + 1], len[g + 1], wn);
      if (T[g] == 0) continue;
      if (T[g] > CB) {
        if (bfill) {
          wave_sync();
          store_group(cb, BUFW, bfill, chars + base + bstart, lane);
          wave_sync();
          bfill = 0;
        }
        if (len[g]) copy_string<gout_u8, gout_u32, true>(sbase, soff + pos[g], chars, base + ex[g], len[g]);
        continue;
      }
      if (bfill + T[g] > CB) {
        wave_sync();
        store_group(cb, BUFW, bfill, chars + base + bstart, lane);
        wave_sync();
        bfill = 0;
      }
      if (bfill == 0) bstart = GB[g];
      if (len[g]) piece_write(wc, sbase, soff + pos[g], cb8, ex[g] - bstart, len[g]);
      bfill += T[g];
    }
    if (bfill) {
      wave_sync();
      store_group(cb, BUFW, bfill, chars + base + bstart, lane);
    }
  }
}

template <bool SLOTS>
__global__ __launch_bounds__(WG) void k_decode_str(uint8_t* __restrict__ ws, const ColScan* __restrict__ cols,
                                                   SegTable seg, uint32_t* __restrict__ err) {
  __shared__ __align__(16) uint32_t s_buf[NWAVES][StrLds<SLOTS>::BUFW];
  WaveTile c;
  if (!wave_tile(seg, cols, ws, c)) return;
  tile_str<SLOTS, false>(c, ws, err, (lds_u32*)&s_buf[threadIdx.x >> 6][0]);
}

// ---------------------------------------------------------------------------
// k_batch: the decode step of a batched scan (many files, requests and
// columns) in one persistent launch.  Each wave takes units (a run of tiles
// of one column with one decoder) from the work queues, its workgroup's home
// queue first (queue i mod NQUEUE for workgroup i, the XCD it is dispatched
// to), then the others in turn, and decodes their tiles one after the other
// with the same tile functions as the one-launch-per-kind form.  REQUIRED
// columns get their validity words here (the work of k_prep); OPTIONAL
// columns' shared edge words are left to k_edges, launched after.  Every
// wave leaves once all NQUEUE queues are drained.
// ---------------------------------------------------------------------------
constexpr uint32_t cmax(uint32_t a, uint32_t b) { return a > b ? a : b; }
constexpr uint32_t BATCH_LDS_WORDS =
    cmax(cmax((uint32_t)PADN, DELTA_LDS_WORDS), cmax(StrLds<true>::BUFW, StrLds<false>::BUFW));

// Validity words of a REQUIRED column whose first row lies in tile c: ones
// for rows below the column's rows, zeros past them (lane j: word j).
__device__ __forceinline__ void tile_required_validity(const WaveTile& c, uint32_t lane) {
  if (c.cs.optional || !c.cs.validity) return;
  const int64_t r0 = c.out0;
  const int64_t W = ((r0 + 31) >> 5) + (int64_t)lane;
  if (lane < 33 && W * 32 < r0 + (int64_t)c.nrows) {
    const int64_t left = c.cs.rows - W * 32;
    reinterpret_cast<uint32_t*>(c.cs.validity)[W] = left >= 32 ? 0xffffffffu : ((1u << left) - 1);
  }
}

__global__ __launch_bounds__(WG) void k_batch(uint8_t* __restrict__ ws, const ColScan* __restrict__ cols,
                                              const BUnit* __restrict__ units, const uint32_t* __restrict__ qbeg,
                                              uint32_t* __restrict__ qhead, uint32_t* __restrict__ err) {
  __shared__ __align__(16) uint32_t s_lds[NWAVES][BATCH_LDS_WORDS];
  lds_u32* wl = (lds_u32*)&s_lds[threadIdx.x >> 6][0];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t home = blockIdx.x % (uint32_t)NQUEUE;
#pragma unroll 1
  for (uint32_t k = 0; k < (uint32_t)NQUEUE; ++k) {
    const uint32_t q = (home + k) % (uint32_t)NQUEUE;
    const uint32_t qb = sload(qbeg + q), qe = sload(qbeg + q + 1);
    if (qb >= qe) continue;
#pragma unroll 1
    for (;;) {
      uint32_t u = 0;
      if (lane == 0) u = atomicAdd(qhead + q, 1u);
      u = qb + (uint32_t)__builtin_amdgcn_readfirstlane((int)u);
      if (u >= qe) break;
      const BUnit bu = sload(units + u);
#pragma unroll 1
      for (uint32_t t = bu.t0; t < bu.t1; ++t) {
        // the column's table is read again for every tile, not held in
        // registers across the loop
        uint32_t csi = bu.cs;
        asm volatile("" : "+s"(csi));
        WaveTile c;
        load_tile(cols, csi, t, ws, c);
        wave_sync();  // the previous tile's LDS reads come first
        switch (bu.kind) {
          case TK_FIXED0: tile_fixed<0, true>(c, ws, err, wl); break;
          case TK_FIXED1: tile_fixed<FX_DICT, true>(c, ws, err, wl); break;
          case TK_FIXED2: tile_fixed<FX_WIDE, true>(c, ws, err, wl); break;
          case TK_FIXED3: tile_fixed<FX_DICT | FX_WIDE, true>(c, ws, err, wl); break;
          case TK_BSS4: tile_fixed<FX_BSS, true>(c, ws, err, wl); break;
          case TK_BSS8: tile_fixed<FX_BSS | FX_WIDE, true>(c, ws, err, wl); break;
          case TK_DELTA: tile_delta<true>(c, ws, err, wl); break;
          case TK_STR: tile_str<false, true>(c, ws, err, wl); break;
          default: tile_str<true, true>(c, ws, err, wl); break;
        }
        tile_required_validity(c, lane);
      }
    }
  }
}

template __global__ void k_decode_str<false>(uint8_t*, const ColScan*, SegTable, uint32_t*);
template __global__ void k_decode_str<true>(uint8_t*, const ColScan*, SegTable, uint32_t*);
template __global__ void k_decode_fixed<0>(uint8_t*, const ColScan*, SegTable, uint32_t*);
template __global__ void k_decode_fixed<FX_DICT>(uint8_t*, const ColScan*, SegTable, uint32_t*);
template __global__ void k_decode_fixed<FX_WIDE>(uint8_t*, const ColScan*, SegTable, uint32_t*);
template __global__ void k_decode_fixed<FX_DICT | FX_WIDE>(uint8_t*, const ColScan*, SegTable, uint32_t*);
template __global__ void k_decode_fixed<FX_BSS>(uint8_t*, const ColScan*, SegTable, uint32_t*);
template __global__ void k_decode_fixed<FX_BSS | FX_WIDE>(uint8_t*, const ColScan*, SegTable, uint32_t*);

}  // namespace pqk
