// pq_internal.h -- data structures shared by the host library and the
// kernels of the GPU scan (chunk table, page table, tile index, per-scan
// column table).
#pragma once
#include <stdint.h>

namespace pqk {

// ---------------------------------------------------------------------------
// format constants (Apache Parquet format description)
// ---------------------------------------------------------------------------
enum : int32_t { T_INT32 = 1, T_INT64 = 2, T_DOUBLE = 5, T_BYTE_ARRAY = 6 };
enum : int32_t { E_PLAIN = 0, E_PLAIN_DICT = 2, E_RLE = 3, E_DELTA = 5, E_DLBA = 6, E_DBA = 7, E_RLE_DICT = 8,
                 E_BSS = 9 };
enum : int32_t { PAGE_DATA = 0, PAGE_INDEX = 1, PAGE_DICT = 2, PAGE_DATA_V2 = 3 };

// device error codes (first error wins; stored as code | (where << 8))
enum : uint32_t {
  ERR_NONE = 0,
  ERR_HEADER = 1,        // page header malformed
  ERR_CHUNK_BOUNDS = 2,  // a page leaves its column chunk
  ERR_PAGE_ORDER = 3,    // dictionary page not first / twice
  ERR_ROWS = 4,          // page value counts do not add up to the row group
  ERR_LEVELS = 5,        // definition-level stream truncated or level > 1
  ERR_VALUES = 6,        // value stream truncated
  ERR_DICT_INDEX = 7,    // dictionary index >= dictionary size
  ERR_DELTA = 8,         // DELTA_BINARY_PACKED header/body invalid
  ERR_SNAPPY = 9,        // Snappy stream invalid
  ERR_UNSUPPORTED = 10,  // encoding / feature outside the supported subset
  ERR_DICT_MISSING = 11, // dictionary-encoded page without a dictionary
  ERR_V2 = 12,           // V2 header inconsistent
  ERR_STRING = 13,       // BYTE_ARRAY length chain invalid
  ERR_CAPACITY = 14      // chars buffer smaller than the decoded strings
};

// Tile = fixed number of rows of one data page.
constexpr int TILE_ROWS = 1024;
// Sub-tile checkpoints: every tile also records, for its level stream at
// every SUB_ROWS-th row and for its dictionary-index stream at every
// SUB_ROWS-th value, the state of the hybrid run holding that row or value,
// so that a scan decodes the pieces of a tile independently and reads the
// payload directly.
//   at:   byte offset from the tile's entry position of the byte holding the
//         value's first bit (bit-packed run), or of the run header (RLE run)
//   info: bit 31 set: bit-packed; bits 28..30 the bit within that byte.
//         RLE runs of a level stream: bit 29 set, bit 30 the level.
//         bits 0..27: values left in the run from this one (clamped).
// DELTA streams record the byte offset of each block header in `at`.
// at == CK_NONE: not recorded (the tile's entry point is used).
constexpr int SUB_ROWS = 64;
constexpr int NSUB = TILE_ROWS / SUB_ROWS;
constexpr uint32_t CK_NONE = 0xffffffffu;
constexpr uint32_t CK_LEFT = 0x0fffffffu;
struct Ck {
  uint32_t at;
  uint32_t info;
};
// Level checkpoints: one word per LROWS rows of a tile (rows 16 l .. 16 l +
// 15 are lane l's), the state of the level run holding that row:
//   bits 0..15   byte offset from the tile's level entry: for a bit-packed run
//                the byte holding the row's bit, for an RLE run the header of
//                the run that follows it
//   bits 16..18  the bit within that byte (bit-packed)
//   bit 19       bit-packed
//   bit 20       the level of an RLE run
//   bits 21..25  values left in the run from this row, at most LROWS
// LCK_NONE: not recorded (offset past 16 bits); the tile's entry is used.
constexpr int LROWS = 16;
constexpr int NLCK = TILE_ROWS / LROWS;
constexpr uint32_t LCK_NONE = 0xffffffffu;
// BYTE_ARRAY checkpoint spacing (values) inside PLAIN string streams and
// string dictionary pages.
constexpr int STR_CK = 32;
// String dictionary pages longer than SCHAIN_MIN bytes have their length
// chain walked at open in SCHAIN_SEG-byte segments side by side (candidate
// chains from each of the first SCHAIN_CAND byte positions of a segment,
// linked segment by segment afterwards); shorter ones by k_index's walk.
constexpr uint32_t SCHAIN_MIN = 256 * 1024;
constexpr uint32_t SCHAIN_SEG = 32768;
constexpr uint32_t SCHAIN_CAND = 64;
constexpr uint32_t SCHAIN_NONE = 0xffffffffu;
struct SChainPage {
  const uint8_t* base;  // buffer holding the page body (the file, or the decompression buffer)
  uint64_t off;         // body offset in base
  uint64_t lim;         // readable bytes of base (a multiple of 16)
  uint32_t len;         // body bytes
  uint32_t n;           // entries
  uint32_t page;        // page index
  uint32_t seg0;        // first segment (in the segment arrays)
  uint32_t nseg;
  uint32_t strck_begin;
};
// A candidate chain of one segment: where it leaves the segment, the
// entries that start in the segment, their longest length, and how it
// ended (0: left the segment; 1: fewer than 4 bytes left; 2: a length past
// the body's end).
struct SChainCand {
  uint32_t exit, count, maxlen, state;
};
// Bytes of slack after every decompressed region (reads run up to 12 bytes
// past a stream end).
constexpr int SCRATCH_PAD = 16;

struct ChunkDev {
  uint64_t start, end;   // byte range of the column chunk in the file
  int64_t rows;          // row-group rows
  int32_t type;          // physical type
  int32_t codec;         // 0 none, 1 snappy
  int32_t optional;
  int32_t col;
};

// Page table entry (one per page, dictionary pages included), in
// column-major chunk order: column 0 rg 0.., column 1 rg 0.., ...
struct PageDev {
  uint64_t payload;      // file offset of the page payload
  uint32_t comp_size;    // compressed_page_size
  uint32_t uncomp_size;  // uncompressed_page_size
  int32_t num_values;    // rows of the page (flat schema); entries for dictionary pages
  int32_t num_nulls;     // V2 header value; -1 for V1
  uint32_t chunk;        // chunk index (col * nrg + rg)
  uint8_t kind;          // PAGE_DATA, PAGE_DICT, PAGE_DATA_V2 (index pages are dropped)
  uint8_t encoding;
  uint8_t v2_compressed; // V2 is_compressed flag (default 1)
  uint8_t flags;         // bit0: level stream in scratch; bit1: value stream in scratch;
                         // bit2: value stream in the expansion region (DELTA_BYTE_ARRAY)
  int32_t def_len;       // level bytes (V2 header; V1 from the body)
  int32_t rep_len;       // V2 header
  uint64_t def_off;      // file offset, or offset inside the page's scratch region
  uint64_t val_off;      // same for the value stream
  uint32_t val_len;
  uint32_t scratch_len;  // decompressed bytes written to scratch (0: not compressed)
  uint64_t scratch_off;  // offset of this page's region in the file-wide scratch layout
  int64_t row0;          // file row of the page's first row
  uint32_t tile_begin;   // first tile of this page
  uint32_t nonnull;      // non-null values (filled by the index pass)
  uint32_t strck_begin;  // first string checkpoint (PLAIN strings / string dictionaries)
  uint32_t dict_page;    // data pages: page index of the chunk's dictionary page (~0u: none)
  // value-stream header facts, parsed once by the index pass:
  //   dictionary pages' data: enc_w = index bit width
  //   DELTA_BINARY_PACKED: enc_w = block size, enc_m = miniblocks,
  //   delta_first = first value, blocks_at = offset of block 0 in the stream
  uint32_t enc_w;
  uint32_t enc_m;
  int64_t delta_first;
  uint32_t blocks_at;
  uint32_t dict_maxlen;  // dictionary pages of strings: length of the longest entry
  uint32_t sblk_begin;   // compressed pages: first entry of the page in the Snappy block index
  uint32_t chars_at;     // DELTA_LENGTH_BYTE_ARRAY pages: value-stream offset of the chars
                         // (the end of the lengths' DELTA_BINARY_PACKED stream)
  // DELTA_BYTE_ARRAY string pages (found by the open-time pass of k_dba):
  // the encoded value stream (x_src: offset in the file, or in the
  // decompression layout when x_scratch), its prefix-length stream from 0,
  // suffix-length stream from x_sfx and suffix bytes from x_chars; the
  // page's values laid out as PLAIN (u32 length + bytes, xlen bytes) at
  // x_off of the expansion layout
  uint64_t x_src;
  uint32_t x_len, x_sfx, x_chars, xlen, x_total, x_scratch;
  uint64_t x_off;
};

// Definition-level streams of OPTIONAL data pages (the levels before the
// values, Sec. 3.3) are hybrid RLE/bit-packed run chains whose run headers
// are only found by walking from the start.  Pages whose body may hold more
// than LV_MIN level bytes are indexed in LV_SEG-byte segments side by side:
// LV_CAND candidate chains per segment (one from each of its first LV_CAND
// bytes), a per-page link through the candidates' exits, then the tile
// entries and level checkpoints per segment.
constexpr uint32_t LV_MIN = 8192;
constexpr uint32_t LV_SEG = 2048;
constexpr uint32_t LV_CAND = 128;
constexpr uint32_t LV_NONE = 0xffffffffu;
__host__ __device__ inline bool lv_page(const PageDev& pg, bool optional) {
  if (!optional || pg.num_values <= 0) return false;
  if (pg.kind == PAGE_DATA) return pg.uncomp_size >= 4u + LV_MIN;  // level bytes <= body - 4
  if (pg.kind == PAGE_DATA_V2) return pg.def_len > (int32_t)LV_MIN;
  return false;
}
struct LvPage {
  uint32_t page, seg0, nseg;  // segments [seg0, seg0 + nseg) of the segment list
};
// A candidate chain of one segment: stream offset where it leaves the
// segment, rows and valid rows of the runs that start in it (saturating at
// 2^32 - 1), and how it ended (0: left the segment or reached the stream end;
// 1: at an invalid run; 2: at a run not held by the staged bytes).
struct LvCand {
  uint32_t exit, state, rows, valid;
};
// The true chain's entry into a segment (stream offset; LV_NONE: the segment
// is not walked) with the rows and valid rows before it.
struct LvEntry {
  uint32_t q, rows, valid, pad_;
};
// DELTA_BINARY_PACKED value streams (and the length streams of
// DELTA_LENGTH_BYTE_ARRAY pages) are chains of blocks whose sizes follow
// from their headers.  Pages whose value stream is longer than DL_MIN bytes
// have the chain walked at open in DL_SEG-byte segments side by side (DL_CAND
// candidate chains per segment, as for level streams); the position of every
// block is stored, and each tile's entry and checkpoints are read from them.
constexpr uint32_t DL_MIN = 16384;
constexpr uint32_t DL_SEG = 16384;
constexpr uint32_t DL_CAND = 256;
__host__ __device__ inline bool dl_page(const PageDev& pg, int32_t type) {
  return pg.kind != PAGE_DICT && pg.num_values > 0 &&
         (pg.encoding == E_DELTA || (pg.encoding == E_DLBA && type == T_BYTE_ARRAY)) && pg.val_len > DL_MIN;
}
struct DlPage {
  uint32_t page, seg0, nseg;  // segments [seg0, seg0 + nseg) of the segment list
  uint32_t blk0;              // first entry of the page in the block-position list
  uint32_t tl0;               // first entry of the page in the tile list
  uint32_t maxw;              // widest miniblock bit width of the column's type
};
// A candidate block chain of one segment: where it leaves the segment, the
// blocks whose header lies in it (every one taken as a full block), and how
// it ended (0: left the segment; 1: at a block that is invalid as a full
// block).
struct DlCand {
  uint32_t exit, count, state, pad_;
};
// The true chain's entry into a segment (value-stream offset; LV_NONE: not
// walked) and the index of the block there.
struct DlEntry {
  uint32_t q, k;
};
// Dictionary-index streams (a bit width byte, then hybrid runs of that
// width) of pages longer than DI_MIN bytes are indexed in DI_SEG-byte
// segments side by side, with di_cand(w) candidate chains per segment: a
// bit-packed run of 63 groups of width w takes 1 + 63 w bytes, so the true
// chain enters a segment within that many bytes of its start (wider runs
// and more than 1024 bytes: the page is walked whole by one wave).
constexpr uint32_t DI_MIN = 16384;
constexpr uint32_t DI_SEG = 32768;
constexpr uint32_t DI_CAND_MAX = 1024;
__host__ __device__ inline bool di_page(const PageDev& pg) {
  return pg.kind != PAGE_DICT && (pg.encoding == E_PLAIN_DICT || pg.encoding == E_RLE_DICT) && pg.num_values > 0 &&
         pg.val_len > DI_MIN;
}
__host__ __device__ inline uint32_t di_cand(uint32_t w) {
  const uint32_t c = (16 + 64 * w + 63) / 64 * 64;
  return c > DI_CAND_MAX ? DI_CAND_MAX : c;
}
struct DiPage {
  uint32_t page, seg0, nseg;  // segments [seg0, seg0 + nseg) of the segment list
  uint32_t tl0;               // first entry of the page in the tile list
};
// A candidate of a dictionary-index stream: where it leaves the segment
// (DI_BAD: at an invalid run) and the values of the runs before (saturating).
constexpr uint32_t DI_BAD = 0xffffffffu;
struct DiCand {
  uint32_t exit, count;
};
// x_total of a DELTA_BYTE_ARRAY page the scan does not decode (a value longer
// than the expansion's LDS buffer, or a DELTA block shape outside the
// supported one): its tiles report PQ_EUNSUPPORTED when its column is scanned
constexpr uint32_t DBA_UNSUPPORTED = 0xffffffffu;
// page encoding given to such a page by the index pass
constexpr uint8_t E_UNDECODED = 0xff;
// Snappy block index: a compressed page's output is cut into SNAP_BLOCK-byte
// blocks; entry b holds the stream offset of the element that starts block
// b.  A page's first entry is SBLK_NONE when some element straddles a block
// boundary or a copy reaches before its block's start: such a page is
// decompressed sequentially, the others one block per lane.
constexpr uint32_t SNAP_BLOCK = 65536;
// k_snappy_blk: blocks decoded per wave; the wave's other lanes only help
// copy long literals.  A wave runs as many batches as its densest block
// needs, so more blocks per wave leave more lanes idle, and fewer leave
// more waves per SIMD: 16 measured best (8, 32 and 64 were slower).
constexpr uint32_t SNAP_LANES = 16;
constexpr uint32_t SBLK_NONE = 0xffffffffu;
// k_snap_order: a scan's blocks in buckets of element count (bucket 0: 8192
// or more, bucket k: [2^(13-k), 2^(14-k)), the last: fewer than 128), the
// densest first, so that the blocks of a k_snappy_blk wave take similar
// numbers of steps.  A bucket entry is (column-table index << 26) | block.
constexpr uint32_t SNAP_BUCKETS = 8;
constexpr uint32_t SNAP_ORD_BITS = 26;

// One tile: rows [row0, row0 + min(TILE_ROWS, num_values - row0)) of page `page`.
struct TileDev {
  uint32_t page;
  uint32_t row0;      // page-relative
  uint32_t k0;        // non-null values before row0 in the page
  uint32_t nn;        // non-null values inside the tile
  uint32_t def_pos;   // level stream: byte offset of the run header holding row0
  uint32_t def_skip;  // values of that run before row0
  uint32_t val_pos;   // value stream entry: run header (dictionary), block header
                      // (DELTA), byte offset of value k0 (PLAIN strings)
  uint32_t val_skip;  // dictionary/DELTA: values of that run/block before k0;
                      // PLAIN strings: byte offset just past the tile's last value
};

// Decoded dictionary of one column chunk, built once when the file is
// opened and kept by the handle (one entry per chunk; n == 0 and page == ~0u
// for a chunk without a dictionary page).  Fixed-width entries are the page
// body itself when it is uncompressed and aligned to the value width, else a
// copy.  String dictionaries keep their body (a copy when the page is
// compressed), (position, length) u32 pairs relative to the body, an array of
// entry lengths (u16 when every entry is shorter than 2^16 bytes, else u32)
// and, when every entry fits SLOT_CHARS bytes, a copy of the entries in fixed
// SLOT_BYTES slots (u32 length first, then the chars, zero-padded), so that
// one row's gather -- length and chars together -- touches one aligned
// 64-byte piece of memory.
constexpr uint32_t SLOT_BYTES = 64;
constexpr uint32_t SLOT_CHARS = 60;
static_assert(SLOT_BYTES == 64 && SLOT_CHARS < 64, "a slot offset and a length share one word");
// Slots are built only for a dictionary that serves at least this many rows
// of its row group per entry: a slot costs 64 bytes of device memory per
// entry for as long as the file is open, which pays only when entries are
// gathered several times.
constexpr uint64_t SLOT_ROWS_PER_ENTRY = 4;
enum : uint32_t { DICT_SLOTS = 1, DICT_LENS16 = 2 };
struct DictSlot {
  const uint8_t* body;   // 16-byte aligned base holding the dictionary page body
  uint64_t body_off;     // offset of the body's first byte from `body`
  uint8_t* entries;      // fixed width: the n entries; strings: (pos, len) u32 pairs
  uint8_t* lens;         // strings: entry lengths
  uint8_t* slots;        // strings with DICT_SLOTS: the slots
  uint32_t n;            // entries (0: chunk has no dictionary)
  uint32_t page;         // dictionary page index (~0u: none)
  uint32_t flags;        // DICT_SLOTS, DICT_LENS16
  int32_t type;          // physical type of the column
};

// Device tables of one opened file, as the kernels of a scan see them (a
// scan over several files carries one copy per selected column).
struct FileDev {
  const uint8_t* file;         // the file bytes (borrowed device buffer)
  const PageDev* pages;        // page table
  const TileDev* tiles;        // tile index
  const uint32_t* ckl;         // level checkpoints, NLCK per tile
  const Ck* ckv;               // value-stream checkpoints, NSUB per tile
  const uint32_t* strck;       // string checkpoints
  const uint64_t* tpfx;        // tile prefix (tiles + 1 entries)
  const uint64_t* tpfx2;       // second tile prefix: DELTA sums of the length streams of
                               // DELTA_LENGTH_BYTE_ARRAY tiles (NULL when the file has none)
  uint32_t* sblk;              // Snappy block index (written by the open-time pass)
  const uint32_t* sblk_page;   // page of each Snappy block
  uint32_t* sblk_ne;           // elements of each Snappy block (written with sblk)
  const DictSlot* dicts;       // resident dictionaries, one per chunk (col * nrg + rg)
};

// Per-scan, per-selected-column table (built on the host, copied into the
// caller's workspace before the kernels run).
struct ColScan {
  FileDev fd;             // the tables of the file this column belongs to
  uint64_t ws_xscratch;   // workspace offset of the expansion region of its DELTA_BYTE_ARRAY pages
  uint64_t xscratch_base; // expansion-layout offset of the region's first byte
  int32_t type;
  int32_t optional;
  int32_t width;          // 4 or 8 (fixed width); 0 for BYTE_ARRAY
  int32_t col;
  uint32_t tile_begin;    // tiles of this column inside the scan: [tile_begin, tile_end)
  uint32_t tile_end;
  uint32_t page_begin;    // pages (incl. dictionary pages) of the scanned chunks
  uint32_t page_end;
  int64_t row_base;       // file row of the scan's first output row
  int64_t rows;           // output rows
  uint64_t scratch_base;  // file-wide scratch offset of this column's first scanned page
  uint64_t ws_scratch;    // workspace offset where this column's decompressed pages start
  uint64_t ws_tile_aux;   // workspace offset of per-tile int64 auxiliaries
  uint64_t chars_capacity;
  void* values;
  uint8_t* validity;
  int64_t* offsets;
  uint8_t* chars;
  uint64_t ws_edge;       // workspace offset of per-tile validity edge words (OPTIONAL columns)
  int32_t open_sel;       // open-time decompression: 0 every page, 1 dictionary pages, 2 data pages
  int32_t pad_;
};
// Whether the open-time decompression pass of ColScan cs takes page pg.
__host__ __device__ inline bool open_sel_ok(const ColScan& cs, const PageDev& pg) {
  return cs.open_sel == 0 || (cs.open_sel == 1) == (pg.kind == PAGE_DICT);
}

// A run of tiles handled by one launch: ColScan `cs`, tiles [t0, t1),
// workgroups [wg0, wg0 + t1 - t0).
struct Segment {
  uint32_t cs, t0, t1, wg0;
};
constexpr int MAX_SEGS = 64;
// With spread set, unit u of the launch is tile u / n of segment u % n (the
// segments' wg0 unused): consecutive waves take tiles of different segments.
struct SegTable {
  Segment s[MAX_SEGS];
  int32_t n;
  int32_t spread;
  const Segment* ptr;  // n > MAX_SEGS: the segments in device memory, ascending in wg0
};

// Batched scans (several files, requests and columns in one launch): every
// unit of work is a run of tiles of one column that one decoder handles.
// The persistent kernel takes units from NQUEUE work queues, queue q first
// for the workgroups dispatched to XCD q (workgroup i runs on XCD i mod 8),
// then the others.
enum : uint32_t { TK_FIXED0 = 0, TK_FIXED1, TK_FIXED2, TK_FIXED3, TK_DELTA, TK_STR, TK_STRSLOT, TK_BSS4, TK_BSS8,
                  TK_KINDS };
struct BUnit {
  uint32_t cs, t0, t1, kind;
};
constexpr int NQUEUE = 8;

// k_dict work (one launch at open for every dictionary page of the file):
// dictionary `slot` (a chunk index) is units [unit0, unit0 + units) of the
// launch, one wave each; the table is ascending in unit0.
struct DictWork {
  uint32_t slot, units, unit0, pad_;
};
// entries per k_dict wave: fixed-width dictionaries; string dictionaries
// take DICT_CK_PER checkpoints of STR_CK entries
constexpr uint32_t DICT_FIXED_PER = 1024;
constexpr uint32_t DICT_CK_PER = 4;

}  // namespace pqk
