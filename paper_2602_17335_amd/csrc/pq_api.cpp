// pq_api.cpp -- host side of the GPU Parquet scan: the C ABI declared in
// include/pq.h.  Footer decode (Thrift compact), page-table and tile-index
// construction at open, workspace planning and kernel orchestration per scan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pq.h"
#include "pq_internal.h"

namespace pqk {
__global__ void k_walk(const uint8_t* file, uint64_t file_lim, const ChunkDev* chunks, int nchunks, uint32_t* counts,
                       const uint32_t* page_base, PageDev* pages, uint32_t* err, uint64_t* rec,
                       const uint32_t* rec_base, const uint32_t* rec_cap, uint32_t* overflow);
__global__ void k_walk_rec(const uint8_t* file, const ChunkDev* chunks, const uint64_t* rec, const uint32_t* rec_base,
                           const uint32_t* page_base, const uint32_t* page_chunk, uint32_t npages, PageDev* pages,
                           uint32_t* err);
__global__ void k_index(const uint8_t* file, const uint8_t* scratch, PageDev* pages, int npages,
                        const ChunkDev* chunks, TileDev* tiles, uint32_t* strck, uint32_t* ckl, Ck* ckv,
                        uint32_t* err, uint64_t file_lim, uint64_t scratch_lim, const uint32_t* order,
                        const uint8_t* xscratch, uint64_t xscratch_lim, int phase);
__global__ void k_lv_cand(const LvPage* lps, const uint32_t* seg_page, const PageDev* pages, const uint8_t* file,
                          const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim, LvCand* cand);
__global__ void k_lv_link(const LvPage* lps, int npg, const PageDev* pages, const LvCand* cand, LvEntry* ent,
                          uint32_t* ok, uint32_t* err);
__global__ void k_lv_tiles(const LvPage* lps, const uint32_t* seg_page, const LvEntry* ent, const uint32_t* ok,
                           PageDev* pages, const uint8_t* file, const uint8_t* scratch, uint64_t file_lim,
                           uint64_t scratch_lim, TileDev* tiles, uint32_t* ckl, uint32_t* err, int mode);
__global__ void k_dl_cand(const DlPage* dps, const uint32_t* seg_page, const PageDev* pages, const uint8_t* file,
                          const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim, DlCand* cand,
                          const uint32_t* err);
__global__ void k_dl_link(const DlPage* dps, int npg, PageDev* pages, const DlCand* cand, DlEntry* ent, uint32_t* ok,
                          uint32_t* err);
__global__ void k_dl_fill(const DlPage* dps, const uint32_t* seg_page, const DlEntry* ent, const uint32_t* ok,
                          PageDev* pages, const uint8_t* file, const uint8_t* scratch, uint64_t file_lim,
                          uint64_t scratch_lim, uint32_t* blkpos, uint32_t* err, int mode);
__global__ void k_dl_tiles(const DlPage* dps, const uint32_t* tile_dp, int ntl, const PageDev* pages, TileDev* tiles,
                           Ck* ckv, const uint32_t* blkpos, const uint32_t* err);
__global__ void k_di_cand(const DiPage* dps, const uint32_t* seg_page, const PageDev* pages, const uint8_t* file,
                          const uint8_t* scratch, uint64_t file_lim, uint64_t scratch_lim, DiCand* cand,
                          const uint32_t* err);
__global__ void k_di_link(const DiPage* dps, int npg, const PageDev* pages, const DiCand* cand, DlEntry* ent,
                          uint32_t* ok, uint32_t* err);
__global__ void k_di_fill(const DiPage* dps, const uint32_t* seg_page, const DlEntry* ent, const uint32_t* ok,
                          const PageDev* pages, const uint8_t* file, const uint8_t* scratch, uint64_t file_lim,
                          uint64_t scratch_lim, TileDev* tiles, uint32_t* err, int mode);
__global__ void k_di_ckpt(const DiPage* dps, const uint32_t* tile_dp, int ntl, const PageDev* pages,
                          const TileDev* tiles, const uint8_t* file, const uint8_t* scratch, uint64_t file_lim,
                          uint64_t scratch_lim, Ck* ckv, const uint32_t* err);
__global__ void k_schain_cand(const SChainPage* pgs, const uint32_t* seg_page, SChainCand* cand);
__global__ void k_schain_link(const SChainPage* pgs, int npg, const SChainCand* cand, uint32_t* seg_start,
                              uint32_t* seg_base, uint32_t* ok);
__global__ void k_schain_fill(const SChainPage* pgs, const uint32_t* seg_page, const uint32_t* seg_start,
                              const uint32_t* seg_base, const uint32_t* ok, uint32_t* strck, PageDev* pages, uint32_t* err);
__global__ void k_schain_seq(const SChainPage* pgs, int npg, const uint32_t* ok, uint32_t* strck, PageDev* pages,
                             uint32_t* err);
__global__ void k_snappy(const ColScan* cols, SegTable seg, uint8_t* ws, int record, uint32_t* err);
__global__ void k_snappy_blk(const ColScan* cols, SegTable seg, const uint32_t* sord, uint32_t cap, uint8_t* ws,
                             uint32_t* err, int dicts);
__global__ void k_snap_order(const ColScan* cols, SegTable seg, uint8_t* ws, uint32_t* sord, uint32_t cap, int mode);
__global__ void k_snap_index(const ColScan* cols, SegTable seg);
__global__ void k_prep(const ColScan* cols, SegTable seg);
__global__ void k_edges(const uint8_t* ws, const ColScan* cols, SegTable seg);
__global__ void k_dict(const PageDev* pages, const uint32_t* strck, const DictSlot* slots, const DictWork* works,
                       uint32_t nworks, uint32_t* err);
__global__ void k_prepass(uint8_t* ws, const ColScan* cols, SegTable seg, int mode, uint32_t* err);
__global__ void k_str_total(const ColScan* cols, const int32_t* which, int32_t n, uint32_t* err);
__global__ void k_copy(uint8_t* dst, const uint8_t* src, uint64_t n);
__global__ void k_dba(const ColScan* cols, SegTable seg, uint8_t* ws, const uint8_t* open_scratch, uint8_t* open_out,
                      PageDev* pages_out, int mode, uint32_t* err);
enum : int { FX_DICT = 1, FX_WIDE = 2, FX_BSS = 4 };
template <int KIND>
__global__ void k_decode_fixed(uint8_t* ws, const ColScan* cols, SegTable seg, uint32_t* err);
__global__ void k_decode_delta(uint8_t* ws, const ColScan* cols, SegTable seg, uint32_t* err);
template <bool SLOTS>
__global__ void k_decode_str(uint8_t* ws, const ColScan* cols, SegTable seg, uint32_t* err);
__global__ void k_batch(uint8_t* ws, const ColScan* cols, const BUnit* units, const uint32_t* qbeg, uint32_t* qhead,
                        uint32_t* err);
}  // namespace pqk

using namespace pqk;

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local char g_msg[512];

static pq_status fail(pq_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static pq_status fail(pq_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return s;
}

#define HIP_OR(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(PQ_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
  } while (0)

extern "C" const char* pq_last_error(void) { return g_msg; }

// ---------------------------------------------------------------------------
// Thrift compact decoder for the footer (host)
// ---------------------------------------------------------------------------
namespace {

struct TReader {
  const uint8_t* p;
  size_t n, pos = 0;
  bool bad = false;
  uint8_t u8() {
    if (pos >= n) { bad = true; return 0; }
    return p[pos++];
  }
  uint64_t uleb() {
    uint64_t v = 0;
    for (int s = 0; s < 70; s += 7) {
      uint8_t b = u8();
      if (bad) return 0;
      if (s == 63 && (b & 0x7e)) { bad = true; return 0; }
      v |= (uint64_t)(b & 0x7f) << s;
      if (!(b & 0x80)) return v;
    }
    bad = true;
    return 0;
  }
  int64_t zz() { uint64_t v = uleb(); return (int64_t)(v >> 1) ^ -(int64_t)(v & 1); }
  // next field of a struct; false at STOP
  bool field(int& last, int& id, int& type) {
    uint8_t b = u8();
    if (bad || b == 0) return false;
    type = b & 15;
    id = (b >> 4) ? last + (b >> 4) : (int)zz();
    last = id;
    return !bad;
  }
  void list_header(uint64_t& size, int& etype) {
    uint8_t b = u8();
    etype = b & 15;
    size = b >> 4;
    if (size == 15) size = uleb();
  }
  void skip(int type, int depth = 0) {
    if (depth > 32) { bad = true; return; }
    switch (type) {
      case 1: case 2: return;
      case 3: u8(); return;
      case 4: case 5: case 6: uleb(); return;
      case 7: if (n - pos < 8) bad = true; else pos += 8; return;
      case 8: { uint64_t l = uleb(); if (bad || l > n - pos) bad = true; else pos += l; return; }
      case 9: case 10: {
        uint64_t sz; int et;
        list_header(sz, et);
        for (uint64_t i = 0; i < sz && !bad; ++i) {
          if (et == 1 || et == 2) u8(); else skip(et, depth + 1);
        }
        return;
      }
      case 11: {
        uint64_t sz = uleb();
        if (!sz) return;
        uint8_t kv = u8();
        for (uint64_t i = 0; i < sz && !bad; ++i) { skip(kv >> 4, depth + 1); skip(kv & 15, depth + 1); }
        return;
      }
      case 12: {
        int last = 0, id, t;
        while (!bad && field(last, id, t)) skip(t, depth + 1);
        return;
      }
      default: bad = true;
    }
  }
};

struct ColMeta {
  int type = 0, optional = 0;
  std::string name;
};
struct ChunkMeta {
  int type = -1, codec = 0;
  int64_t num_values = -1, total_compressed = -1, data_off = -1, dict_off = -1;
  bool has_dict = false, external = false;
};

pq_status parse_footer(const uint8_t* p, size_t n, std::vector<ColMeta>& cols, std::vector<int64_t>& rg_rows,
                       std::vector<ChunkMeta>& chunks /* [rg][col] */) {
  TReader r{p, n};
  int last = 0, id, t;
  bool have_schema = false, have_rgs = false;
  while (r.field(last, id, t)) {
    if (id == 2 && t == 9) {
      uint64_t sz; int et;
      r.list_header(sz, et);
      if (r.bad || et != 12 || sz < 1) return fail(PQ_ECORRUPT, "bad schema list");
      for (uint64_t e = 0; e < sz; ++e) {
        int l2 = 0, i2, t2, type = -1, rep = 0, nch = 0;
        std::string name;
        while (r.field(l2, i2, t2)) {
          if (i2 == 1 && t2 == 5) type = (int)r.zz();
          else if (i2 == 3 && t2 == 5) rep = (int)r.zz();
          else if (i2 == 5 && t2 == 5) nch = (int)r.zz();
          else if (i2 == 4 && t2 == 8) {
            uint64_t l = r.uleb();
            if (r.bad || l > r.n - r.pos) return fail(PQ_ECORRUPT, "bad schema name");
            name.assign((const char*)r.p + r.pos, l);
            r.pos += l;
          } else r.skip(t2);
        }
        if (r.bad) return fail(PQ_ECORRUPT, "bad schema element");
        if (e == 0) {
          if ((uint64_t)nch != sz - 1) return fail(PQ_EUNSUPPORTED, "nested schemas are not supported");
          continue;
        }
        if (nch != 0 || type < 0) return fail(PQ_EUNSUPPORTED, "nested schemas are not supported");
        if (rep == 2) return fail(PQ_EUNSUPPORTED, "REPEATED columns are not supported");
        if (type != T_INT32 && type != T_INT64 && type != T_DOUBLE && type != T_BYTE_ARRAY)
          return fail(PQ_EUNSUPPORTED, "column %s: physical type %d is not supported", name.c_str(), type);
        ColMeta c;
        c.type = type;
        c.optional = rep == 1;
        c.name = name;
        cols.push_back(c);
      }
      have_schema = true;
    } else if (id == 4 && t == 9) {
      uint64_t nrg; int et;
      r.list_header(nrg, et);
      if (r.bad || et != 12 || !have_schema) return fail(PQ_ECORRUPT, "bad row-group list");
      for (uint64_t g = 0; g < nrg; ++g) {
        int l2 = 0, i2, t2;
        int64_t rows = -1;
        bool have_cols = false;
        while (r.field(l2, i2, t2)) {
          if (i2 == 1 && t2 == 9) {
            uint64_t nc; int e2;
            r.list_header(nc, e2);
            if (r.bad || e2 != 12 || nc != cols.size()) return fail(PQ_ECORRUPT, "row group column count mismatch");
            for (uint64_t c = 0; c < nc; ++c) {
              ChunkMeta cm;
              int l3 = 0, i3, t3;
              while (r.field(l3, i3, t3)) {
                if (i3 == 1 && t3 == 8) { cm.external = true; r.skip(t3); }
                else if (i3 == 3 && t3 == 12) {
                  int l4 = 0, i4, t4;
                  while (r.field(l4, i4, t4)) {
                    if (i4 == 1 && t4 == 5) cm.type = (int)r.zz();
                    else if (i4 == 4 && t4 == 5) cm.codec = (int)r.zz();
                    else if (i4 == 5 && t4 == 6) cm.num_values = r.zz();
                    else if (i4 == 7 && t4 == 6) cm.total_compressed = r.zz();
                    else if (i4 == 9 && t4 == 6) cm.data_off = r.zz();
                    else if (i4 == 11 && t4 == 6) { cm.dict_off = r.zz(); cm.has_dict = true; }
                    else r.skip(t4);
                  }
                } else r.skip(t3);
              }
              chunks.push_back(cm);
            }
            have_cols = true;
          } else if (i2 == 3 && t2 == 6) rows = r.zz();
          else r.skip(t2);
        }
        if (r.bad || !have_cols || rows < 0) return fail(PQ_ECORRUPT, "bad row group");
        rg_rows.push_back(rows);
      }
      have_rgs = true;
    } else {
      r.skip(t);
    }
    if (r.bad) break;
  }
  if (r.bad || !have_schema || !have_rgs) return fail(PQ_ECORRUPT, "malformed file metadata");
  return PQ_OK;
}

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
constexpr int NKERN = 18;  // kernels with a profiling slot (each fixed-width instantiation has its own)

struct pq_file_s {
  const uint8_t* file = nullptr;  // the device-resident file (NULL for a host-resident one)
  const uint8_t* host = nullptr;  // a host-resident file (pq_open_host), borrowed
  uint64_t len = 0;
  int ncols = 0, nrg = 0;
  std::vector<ColMeta> cols;
  std::vector<int64_t> rg_rows, rg_row0;
  std::vector<ChunkDev> chunks;          // col-major
  std::vector<uint32_t> chunk_page0;     // first page of each chunk (+ sentinel)
  std::vector<uint32_t> chunk_tile0;     // first tile of each chunk (+ sentinel)
  std::vector<PageDev> pages;            // host copy (after the index pass)
  std::vector<uint64_t> scratch_prefix;  // per page (+ sentinel): file-wide scratch offset
  std::vector<uint64_t> xscratch_prefix; // per page (+ sentinel): expansion-layout offset (DELTA_BYTE_ARRAY pages)
  uint64_t total_tiles = 0, total_strck = 0;
  PageDev* d_pages = nullptr;
  TileDev* d_tiles = nullptr;
  uint32_t* d_strck = nullptr;
  uint32_t* d_sblk = nullptr;       // Snappy block index (stream offset per 64 KiB output block)
  uint32_t* d_sblk_page = nullptr;  // page of each block
  uint64_t total_sblk = 0;
  uint32_t* d_ckl = nullptr;  // level checkpoints, NLCK per tile
  Ck* d_ckv = nullptr;  // value-stream checkpoints, NSUB per tile
  ChunkDev* d_chunks = nullptr;
  uint32_t* d_err = nullptr;
  // tile prefix: exclusive prefix sum over the file's tiles of each tile's
  // DELTA sum or string byte count (total_tiles + 1 entries), on the device
  // and on the host
  uint64_t* d_tpfx = nullptr;
  std::vector<uint64_t> tpfx;
  uint64_t* d_tpfx2 = nullptr;  // second tile prefix (DELTA_LENGTH_BYTE_ARRAY length streams)
  // resident dictionaries: one DictSlot per chunk (device and host), their
  // decoded arrays in one arena
  DictSlot* d_dicts = nullptr;
  uint8_t* d_dict_arena = nullptr;
  std::vector<DictSlot> dicts;
  uint64_t device_bytes = 0;  // device memory held by the handle
  FileDev fd{};               // the device tables, as a scan's columns carry them
  pq_file_stats stats{};
  // measurement hook: event pairs around each launched kernel
  bool profiling = false;
  struct Rec { int kernel; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  // pq_scan_streamed: per staging slot, "copied" and "free again" events
  hipEvent_t stage_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  double prof_ms[NKERN] = {0};
  uint64_t prof_n[NKERN] = {0};
};

// Slot order; k_decode_fixed<K> for K = 0 PLAIN 4-byte, 1 dictionary 4-byte,
// 2 PLAIN 8-byte, 3 dictionary 8-byte; k_decode_str<true> decodes the tiles
// of slot dictionaries, k_decode_str<false> the others.
enum { KP_SNAPPY, KP_DICT, KP_STR_TOTAL, KP_PREP, KP_FIXED0, KP_STR = KP_FIXED0 + 8, KP_DELTA, KP_EDGES,
       KP_STR_SLOTS, KP_SNAPPY_BLK, KP_BATCH };
static const char* kKernelNames[NKERN] = {"k_snappy", "k_dict", "k_str_total", "k_prep",
                                          "k_decode_fixed<0>", "k_decode_fixed<1>", "k_decode_fixed<2>",
                                          "k_decode_fixed<3>", "k_decode_fixed<4>", "k_decode_fixed<5>",
                                          "k_decode_fixed<6>", "k_decode_fixed<7>", "k_decode_str<false>",
                                          "k_decode_delta", "k_edges", "k_decode_str<true>", "k_snappy_blk", "k_batch"};

static hipEvent_t pool_get(pq_file f) {
  if (!f->event_pool.empty()) {
    hipEvent_t e = f->event_pool.back();
    f->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
  pq_file f;
  int k;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(pq_file f_, int k_, hipStream_t s_) : f(f_), k(k_), s(s_) {
    if (f->profiling) {
      a = pool_get(f);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = pool_get(f);
    if (!b) return;
    (void)hipEventRecord(b, s);
    f->recs.push_back(pq_file_s::Rec{k, a, b});
  }
};

static void free_handle(pq_file f) {
  if (!f) return;
  for (auto& r : f->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : f->event_pool) (void)hipEventDestroy(e);
  for (auto e : f->stage_ev)
    if (e) (void)hipEventDestroy(e);
  if (f->d_pages) (void)hipFree(f->d_pages);
  if (f->d_tiles) (void)hipFree(f->d_tiles);
  if (f->d_strck) (void)hipFree(f->d_strck);
  if (f->d_sblk) (void)hipFree(f->d_sblk);
  if (f->d_sblk_page) (void)hipFree(f->d_sblk_page);
  if (f->d_ckl) (void)hipFree(f->d_ckl);
  if (f->d_ckv) (void)hipFree(f->d_ckv);
  if (f->d_chunks) (void)hipFree(f->d_chunks);
  if (f->d_err) (void)hipFree(f->d_err);
  if (f->d_tpfx) (void)hipFree(f->d_tpfx);
  if (f->d_tpfx2) (void)hipFree(f->d_tpfx2);
  if (f->d_dicts) (void)hipFree(f->d_dicts);
  if (f->d_dict_arena) (void)hipFree(f->d_dict_arena);
  delete f;
}

static pq_status device_error(uint32_t code) {
  const uint32_t c = code & 0xff, where = code >> 8;
  static const char* names[] = {"none", "page header", "page leaves its column chunk", "page order",
                                "page value counts", "definition levels", "value stream", "dictionary index",
                                "DELTA_BINARY_PACKED data", "Snappy stream", "unsupported feature",
                                "dictionary missing", "V2 page header", "BYTE_ARRAY lengths", "chars capacity"};
  const char* nm = c < sizeof(names) / sizeof(names[0]) ? names[c] : "?";
  if (c == ERR_UNSUPPORTED) return fail(PQ_EUNSUPPORTED, "device: unsupported feature (at %u)", where);
  if (c == ERR_CAPACITY) return fail(PQ_ECAPACITY, "device: chars buffer too small (column %u)", where);
  return fail(PQ_ECORRUPT, "device: corrupt %s (at %u)", nm, where);
}

// Reads (and on error clears) a device error word after synchronising s.
static pq_status read_err_word(uint32_t* d_word, hipStream_t s) {
  uint32_t e = 0;
  HIP_OR(hipMemcpyAsync(&e, d_word, 4, hipMemcpyDeviceToHost, s));
  HIP_OR(hipStreamSynchronize(s));
  if (e) {
    HIP_OR(hipMemsetAsync(d_word, 0, 4, s));
    HIP_OR(hipStreamSynchronize(s));
    return device_error(e);
  }
  return PQ_OK;
}
static pq_status read_err(pq_file f, hipStream_t s) { return read_err_word(f->d_err, s); }

static SegTable make_segs(const std::vector<Segment>& v, bool spread = false) {
  SegTable t;
  memset(&t, 0, sizeof(t));
  t.n = (int32_t)v.size();
  t.spread = spread ? 1 : 0;
  for (size_t i = 0; i < v.size(); ++i) t.s[i] = v[i];
  return t;
}

static pq_status build_tile_prefix(pq_file f, hipStream_t s);
static pq_status build_dicts(pq_file f, const uint8_t* scratch, bool copy_all, hipStream_t s);

// Decompressed bytes of the data pages indexed together at open.
constexpr uint64_t OPEN_SCRATCH_CAP = 512ull << 20;
// Bytes allocated before an open-time window: the index walks' stream
// readers fill their LDS windows from up to 256 bytes before the position
// they move to, which for a pass's first page lies before the window.
constexpr uint64_t OPEN_GUARD = 4096;

// The open of a file in device memory; with host_copy the buffer is a
// temporary device copy of a host-resident file, so every dictionary is
// copied into the handle's arena (none may point into the buffer).
static pq_status open_impl(const void* dev_buf, uint64_t len, pq_stream stream, bool host_copy, pq_file* out) {
  if (!out) return fail(PQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (!dev_buf) return fail(PQ_EINVAL, "dev_buf is NULL");
  if (((uintptr_t)dev_buf & 15) != 0) return fail(PQ_EINVAL, "dev_buf must be 16-byte aligned");
  if (len < 12) return fail(PQ_ECORRUPT, "file shorter than 12 bytes");
  hipStream_t s = (hipStream_t)stream;
  auto t0 = std::chrono::steady_clock::now();
  const uint8_t* file = (const uint8_t*)dev_buf;
  uint8_t tail[8], head[4];
  HIP_OR(hipMemcpyAsync(tail, file + len - 8, 8, hipMemcpyDeviceToHost, s));
  HIP_OR(hipMemcpyAsync(head, file, 4, hipMemcpyDeviceToHost, s));
  HIP_OR(hipStreamSynchronize(s));
  if (memcmp(tail + 4, "PAR1", 4) || memcmp(head, "PAR1", 4)) return fail(PQ_ECORRUPT, "bad magic");
  uint64_t flen = (uint64_t)tail[0] | ((uint64_t)tail[1] << 8) | ((uint64_t)tail[2] << 16) | ((uint64_t)tail[3] << 24);
  if (flen + 12 > len) return fail(PQ_ECORRUPT, "footer length exceeds file");
  std::vector<uint8_t> foot(flen);
  if (flen) {
    HIP_OR(hipMemcpyAsync(foot.data(), file + len - 8 - flen, flen, hipMemcpyDeviceToHost, s));
    HIP_OR(hipStreamSynchronize(s));
  }
  pq_file f = new pq_file_s();
  f->file = file;
  f->len = len;
  std::vector<ChunkMeta> cms;
  pq_status st = parse_footer(foot.data(), foot.size(), f->cols, f->rg_rows, cms);
  if (st != PQ_OK) { free_handle(f); return st; }
  f->ncols = (int)f->cols.size();
  f->nrg = (int)f->rg_rows.size();
  if (f->ncols > 64) { free_handle(f); return fail(PQ_EUNSUPPORTED, "more than 64 columns"); }
  f->rg_row0.resize(f->nrg + 1, 0);
  for (int g = 0; g < f->nrg; ++g) f->rg_row0[g + 1] = f->rg_row0[g] + f->rg_rows[g];
  const uint64_t data_end = len - 8 - flen;
  const int nchunks = f->ncols * f->nrg;
  f->chunks.resize(nchunks);
  for (int c = 0; c < f->ncols; ++c)
    for (int g = 0; g < f->nrg; ++g) {
      const ChunkMeta& m = cms[(size_t)g * f->ncols + c];
      if (m.external) { free_handle(f); return fail(PQ_EUNSUPPORTED, "column chunk in another file"); }
      if (m.type != f->cols[c].type) { free_handle(f); return fail(PQ_ECORRUPT, "chunk type differs from schema"); }
      if (m.codec != 0 && m.codec != 1) { free_handle(f); return fail(PQ_EUNSUPPORTED, "codec %d is not supported", m.codec); }
      if (m.num_values != f->rg_rows[g]) { free_handle(f); return fail(PQ_ECORRUPT, "chunk value count differs from row-group rows"); }
      int64_t start = m.data_off;
      if (m.has_dict && m.dict_off > 0 && m.dict_off < m.data_off) start = m.dict_off;
      if (start < 4 || m.total_compressed < 0 || (uint64_t)start + (uint64_t)m.total_compressed > data_end) {
        free_handle(f);
        return fail(PQ_ECORRUPT, "column chunk outside the file");
      }
      ChunkDev& cd = f->chunks[(size_t)c * f->nrg + g];
      cd.start = (uint64_t)start;
      cd.end = (uint64_t)start + (uint64_t)m.total_compressed;
      cd.rows = f->rg_rows[g];
      cd.type = m.type;
      cd.codec = m.codec;
      cd.optional = f->cols[c].optional;
      cd.col = c;
    }

  // ---- a2: device page-header walk ----
  hipEvent_t e0, e1;
  HIP_OR(hipEventCreate(&e0));
  HIP_OR(hipEventCreate(&e1));
  HIP_OR(hipEventRecord(e0, s));
  uint32_t *d_counts = nullptr, *d_base = nullptr;
  uint8_t* d_rec = nullptr;  // header offsets recorded by the first walk, with their tables
  auto cleanup_tmp = [&]() {
    if (d_counts) (void)hipFree(d_counts);
    if (d_base) (void)hipFree(d_base);
    if (d_rec) (void)hipFree(d_rec);
    d_counts = d_base = nullptr;
    d_rec = nullptr;
  };
#define OPEN_HIP(expr)                                                          \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      cleanup_tmp();                                                            \
      free_handle(f);                                                           \
      return fail(PQ_EHIP, "%s: %s", #expr, hipGetErrorString(e_));            \
    }                                                                           \
  } while (0)
#define OPEN_ERR()                                                              \
  do {                                                                          \
    pq_status st_ = read_err(f, s);                                             \
    if (st_ != PQ_OK) { cleanup_tmp(); free_handle(f); return st_; }            \
  } while (0)

  OPEN_HIP(hipMalloc(&f->d_err, 4));
  OPEN_HIP(hipMemsetAsync(f->d_err, 0, 4, s));
  // The first walk checks every header, counts the pages and records the
  // header offsets of up to one page per KiB of each chunk; the page table
  // is then parsed from the recorded offsets side by side, or, when a chunk
  // has more pages than recorded, by a second walk.
  std::vector<uint32_t> rec_base(nchunks + 1, 0), rec_cap(nchunks);
  for (int q = 0; q < nchunks; ++q) {
    rec_cap[q] = (uint32_t)std::min<uint64_t>((f->chunks[q].end - f->chunks[q].start) / 1024 + 8, 1u << 24);
    rec_base[q + 1] = rec_base[q] + rec_cap[q];
  }
  const size_t o_rbase = align_up(8ull * rec_base[nchunks], 256), o_rcap = align_up(o_rbase + 4ull * nchunks, 256),
               o_over = align_up(o_rcap + 4ull * nchunks, 256), o_pch = align_up(o_over + 4, 256);
  uint32_t overflow = 1;
  if (nchunks > 0) {
    OPEN_HIP(hipMalloc(&f->d_chunks, sizeof(ChunkDev) * nchunks));
    OPEN_HIP(hipMalloc(&d_counts, sizeof(uint32_t) * nchunks));
    OPEN_HIP(hipMalloc(&d_base, sizeof(uint32_t) * nchunks));
    OPEN_HIP(hipMemcpyAsync(f->d_chunks, f->chunks.data(), sizeof(ChunkDev) * nchunks, hipMemcpyHostToDevice, s));
    const bool record = hipMalloc(&d_rec, o_pch) == hipSuccess;  // (no room: the second walk)
    uint64_t* d_recs = record ? reinterpret_cast<uint64_t*>(d_rec) : nullptr;
    uint32_t* d_rbase = record ? reinterpret_cast<uint32_t*>(d_rec + o_rbase) : nullptr;
    uint32_t* d_rcap = record ? reinterpret_cast<uint32_t*>(d_rec + o_rcap) : nullptr;
    uint32_t* d_over = record ? reinterpret_cast<uint32_t*>(d_rec + o_over) : nullptr;
    if (record) {
      OPEN_HIP(hipMemcpyAsync(d_rbase, rec_base.data(), 4ull * nchunks, hipMemcpyHostToDevice, s));
      OPEN_HIP(hipMemcpyAsync(d_rcap, rec_cap.data(), 4ull * nchunks, hipMemcpyHostToDevice, s));
      OPEN_HIP(hipMemsetAsync(d_over, 0, 4, s));
    }
    hipLaunchKernelGGL(k_walk, dim3((uint32_t)nchunks), dim3(64), 0, s, file, (len + 15) & ~15ull, f->d_chunks, nchunks,
                       d_counts, nullptr, nullptr, f->d_err, d_recs, d_rbase, d_rcap, d_over);
    OPEN_HIP(hipGetLastError());
    OPEN_ERR();
    if (record) OPEN_HIP(hipMemcpy(&overflow, d_over, 4, hipMemcpyDeviceToHost));
  }
  std::vector<uint32_t> counts(nchunks);
  if (nchunks) OPEN_HIP(hipMemcpy(counts.data(), d_counts, sizeof(uint32_t) * nchunks, hipMemcpyDeviceToHost));
  f->chunk_page0.assign(nchunks + 1, 0);
  for (int q = 0; q < nchunks; ++q) f->chunk_page0[q + 1] = f->chunk_page0[q] + counts[q];
  const uint32_t npages = f->chunk_page0[nchunks];
  if (npages > 0) {
    OPEN_HIP(hipMalloc(&f->d_pages, sizeof(PageDev) * npages));
    OPEN_HIP(hipMemcpyAsync(d_base, f->chunk_page0.data(), sizeof(uint32_t) * nchunks, hipMemcpyHostToDevice, s));
    uint32_t* d_pch = nullptr;
    std::vector<uint32_t> page_chunk;
    if (!overflow) {
      page_chunk.resize(npages);
      for (int q = 0; q < nchunks; ++q)
        for (uint32_t p = f->chunk_page0[q]; p < f->chunk_page0[q + 1]; ++p) page_chunk[p] = (uint32_t)q;
      if (hipMalloc(&d_pch, 4ull * npages) != hipSuccess) overflow = 1;
    }
    if (!overflow) {
      hipError_t e2 = hipMemcpyAsync(d_pch, page_chunk.data(), 4ull * npages, hipMemcpyHostToDevice, s);
      if (e2 == hipSuccess) {
        hipLaunchKernelGGL(k_walk_rec, dim3((npages + 255) / 256), dim3(256), 0, s, file, f->d_chunks,
                           reinterpret_cast<const uint64_t*>(d_rec), reinterpret_cast<const uint32_t*>(d_rec + o_rbase),
                           d_base, d_pch, npages, f->d_pages, f->d_err);
        e2 = hipGetLastError();
      }
      if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);  // before d_pch and page_chunk go
      (void)hipFree(d_pch);
      OPEN_HIP(e2);
    } else {
      hipLaunchKernelGGL(k_walk, dim3((uint32_t)nchunks), dim3(64), 0, s, file, (len + 15) & ~15ull, f->d_chunks,
                         nchunks, nullptr, d_base, f->d_pages, f->d_err, nullptr, nullptr, nullptr, nullptr);
      OPEN_HIP(hipGetLastError());
    }
    OPEN_ERR();
    f->pages.resize(npages);
    OPEN_HIP(hipMemcpy(f->pages.data(), f->d_pages, sizeof(PageDev) * npages, hipMemcpyDeviceToHost));
  }
  cleanup_tmp();

  // ---- host layout: rows, dictionary links, tiles, scratch, checkpoints ----
  f->chunk_tile0.assign(nchunks + 1, 0);
  f->scratch_prefix.assign(npages + 1, 0);
  uint64_t tiles = 0, strck = 0, scratch = 0, sblk = 0;
  std::vector<uint32_t> sblk_page;
  for (int q = 0; q < nchunks; ++q) {
    const ChunkDev& cd = f->chunks[q];
    const int g = q % f->nrg;
    int64_t row = f->rg_row0[g];
    uint32_t dict = ~0u;
    f->chunk_tile0[q] = (uint32_t)tiles;
    for (uint32_t p = f->chunk_page0[q]; p < f->chunk_page0[q + 1]; ++p) {
      PageDev& pg = f->pages[p];
      pg.scratch_off = scratch;  // (dictionary pages: placed after the data pages below)
      f->scratch_prefix[p] = scratch;
      uint64_t slen = 0;
      if (cd.codec == 1) {
        if (pg.kind == PAGE_DATA_V2) slen = pg.v2_compressed ? pg.uncomp_size - pg.rep_len - pg.def_len : 0;
        else slen = pg.uncomp_size;
        // V1/dictionary pages are always compressed with the chunk codec; an
        // empty page still decompresses to 0 bytes
        if (slen == 0 && pg.kind != PAGE_DATA_V2) slen = 0;
      }
      pg.scratch_len = (uint32_t)slen;
      pg.sblk_begin = (uint32_t)sblk;
      if (slen) {
        const uint64_t nb = (slen + SNAP_BLOCK - 1) / SNAP_BLOCK;
        for (uint64_t j = 0; j < nb; ++j) sblk_page.push_back(p);
        sblk += nb;
      }
      if (cd.codec == 1 && (pg.kind != PAGE_DATA_V2 || pg.v2_compressed) && pg.kind != PAGE_DICT)
        scratch += align_up(slen + SCRATCH_PAD, 16);
      if (pg.kind == PAGE_DICT) {
        dict = p;
        pg.row0 = row;
        if (cd.type == T_BYTE_ARRAY) {
          pg.strck_begin = (uint32_t)strck;
          strck += (uint64_t)pg.num_values / STR_CK + 1;
        }
        continue;
      }
      pg.dict_page = dict;
      pg.row0 = row;
      row += pg.num_values;
      pg.tile_begin = (uint32_t)tiles;
      tiles += ((uint64_t)pg.num_values + TILE_ROWS - 1) / TILE_ROWS;
      if (cd.type == T_BYTE_ARRAY && (pg.encoding == E_PLAIN || pg.encoding == E_DBA)) {
        pg.strck_begin = (uint32_t)strck;
        strck += (uint64_t)pg.num_values / STR_CK + 1;
      }
    }
  }
  f->chunk_tile0[nchunks] = (uint32_t)tiles;
  f->scratch_prefix[npages] = scratch;
  // the scratch layout: data pages in page order (a scan decompresses a
  // column's data pages into one range), then the dictionary pages, which
  // are decompressed at open only
  uint64_t dict_scratch = 0;
  for (uint32_t p = 0; p < npages; ++p) {
    PageDev& pg = f->pages[p];
    if (pg.kind != PAGE_DICT) continue;
    pg.scratch_off = scratch + dict_scratch;
    if (f->chunks[pg.chunk].codec == 1) dict_scratch += align_up((uint64_t)pg.scratch_len + SCRATCH_PAD, 16);
  }
  f->xscratch_prefix.assign(npages + 1, 0);
  if (tiles > 0xffffffffull) { free_handle(f); return fail(PQ_EUNSUPPORTED, "too many tiles"); }
  f->total_tiles = tiles;
  f->total_strck = strck;

  // ---- the index passes ----
  // Compressed pages are decompressed for the index in passes, each into one
  // window: first every dictionary page (their region follows the data
  // pages' in the scratch layout), then the data pages in runs of
  // consecutive pages whose decompressed bytes fit OPEN_SCRATCH_CAP (a larger
  // page is a run of its own).  The kernels of a pass address the window
  // through the file-wide scratch offsets, shifted by the pass's first one.
  struct OpenPass { bool dict; uint32_t p0, p1; uint64_t s0, s1; };
  std::vector<OpenPass> passes;
  passes.push_back(OpenPass{true, 0, npages, scratch, scratch + dict_scratch});
  for (uint32_t p = 0; p < npages;) {
    uint32_t p1 = p + 1;
    const uint64_t a = f->scratch_prefix[p];
    while (p1 < npages && f->scratch_prefix[p1 + 1] - a <= OPEN_SCRATCH_CAP) ++p1;
    passes.push_back(OpenPass{false, p, p1, a, f->scratch_prefix[p1]});
    p = p1;
  }
  uint64_t window = 0;
  for (const OpenPass& P : passes) window = std::max(window, P.s1 - P.s0);
  uint8_t* d_scratch_mem = nullptr;  // the window, after OPEN_GUARD bytes
  uint8_t* d_scratch = nullptr;
  ColScan* d_cs = nullptr;
  uint32_t* d_order = nullptr;
  uint8_t* d_schain = nullptr;  // long string dictionaries: segment tables of the chain walk
  uint8_t* d_lv = nullptr;      // long level streams: segment tables of their walk
  uint8_t* d_dl = nullptr;      // long DELTA streams: segment, block and tile tables of their walk
  uint8_t* d_di = nullptr;      // long dictionary-index streams: segment and tile tables of their walk
  uint8_t* d_xscratch_mem = nullptr;  // DELTA_BYTE_ARRAY pages of a pass expanded to the PLAIN layout,
  uint8_t* d_xscratch = nullptr;      // after OPEN_GUARD bytes
  ColScan* d_xcols = nullptr;     // their column tables
  uint64_t xscratch = 0;          // bytes of the file-wide expansion layout so far
  auto free_pass = [&]() {
    if (d_order) (void)hipFree(d_order);
    if (d_schain) (void)hipFree(d_schain);
    if (d_lv) (void)hipFree(d_lv);
    if (d_dl) (void)hipFree(d_dl);
    if (d_di) (void)hipFree(d_di);
    if (d_xscratch_mem) (void)hipFree(d_xscratch_mem);
    if (d_xcols) (void)hipFree(d_xcols);
    d_order = nullptr;
    d_schain = nullptr;
    d_lv = nullptr;
    d_dl = nullptr;
    d_di = nullptr;
    d_xscratch_mem = d_xscratch = nullptr;
    d_xcols = nullptr;
  };
  auto cleanup_open = [&]() {
    free_pass();
    if (d_scratch_mem) (void)hipFree(d_scratch_mem);
    if (d_cs) (void)hipFree(d_cs);
    d_scratch_mem = d_scratch = nullptr;
    d_cs = nullptr;
  };
  if (npages) OPEN_HIP(hipMemcpyAsync(f->d_pages, f->pages.data(), sizeof(PageDev) * npages, hipMemcpyHostToDevice, s));
  // Snappy block index, built by the decompression below
  f->total_sblk = sblk;
  if (sblk) {
    if (hipMalloc(&f->d_sblk, 2 * sizeof(uint32_t) * sblk) != hipSuccess ||  // offsets, then element counts
        hipMalloc(&f->d_sblk_page, sizeof(uint32_t) * sblk) != hipSuccess) {
      cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: block index allocation");
    }
    if (hipMemcpy(f->d_sblk_page, sblk_page.data(), sizeof(uint32_t) * sblk, hipMemcpyHostToDevice) != hipSuccess) {
      cleanup_open(); free_handle(f); return fail(PQ_EHIP, "open: block index upload");
    }
  }
  if (window > 0) {
    if (hipMalloc(&d_scratch_mem, OPEN_GUARD + window) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: no device memory for decompression"); }
    d_scratch = d_scratch_mem + OPEN_GUARD;
  }
  if (hipMalloc(&d_cs, sizeof(ColScan)) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: allocation failed"); }
  if (tiles) {
    if (hipMalloc(&f->d_tiles, sizeof(TileDev) * tiles) != hipSuccess ||
        hipMalloc(&f->d_ckl, sizeof(uint32_t) * NLCK * tiles) != hipSuccess ||
        hipMalloc(&f->d_ckv, sizeof(Ck) * NSUB * tiles) != hipSuccess) {
      cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: tile index allocation");
    }
  }
  if (strck) {
    if (hipMalloc(&f->d_strck, sizeof(uint32_t) * strck) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: checkpoint allocation"); }
  }
  const uint64_t flim = (len + 15) & ~15ull;  // the file is readable up to len rounded up to 16
  if (sblk) {
    // the Snappy block index of every compressed page, from a walk over the
    // element tags (it reads the compressed pages only, so one launch serves
    // every pass)
    ColScan cs;
    memset(&cs, 0, sizeof(cs));
    cs.fd.file = file;
    cs.fd.pages = f->d_pages;
    cs.fd.sblk = f->d_sblk;
    cs.fd.sblk_page = f->d_sblk_page;
    cs.fd.sblk_ne = f->d_sblk + f->total_sblk;
    OPEN_HIP(hipMemcpyAsync(d_cs, &cs, sizeof(cs), hipMemcpyHostToDevice, s));
    std::vector<Segment> segs{Segment{0, 0, npages, 0}};
    hipLaunchKernelGGL(k_snap_index, dim3(npages), dim3(64), 0, s, d_cs, make_segs(segs));
    if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_snap_index launch failed"); }
  }
  for (const OpenPass& P : passes) {
    // this pass's pages; scr + (file-wide scratch offset) addresses the window
    std::vector<uint32_t> plist;
    bool any_comp = false;
    for (uint32_t p = P.p0; p < P.p1; ++p)
      if ((f->pages[p].kind == PAGE_DICT) == P.dict) {
        plist.push_back(p);
        any_comp |= f->pages[p].scratch_len > 0;
      }
    const uint8_t* scr = d_scratch ? d_scratch - P.s0 : nullptr;
    const uint64_t scr_lim = P.s1;
    const uint8_t* xscr = nullptr;  // the pass's expansion region, addressed through the file-wide layout
    uint64_t xscr_lim = 0;
    if (any_comp) {
      // the indexed blocks side by side, the other pages one wave each
      ColScan cs;
      memset(&cs, 0, sizeof(cs));
      cs.fd.file = file;
      cs.fd.pages = f->d_pages;
      cs.fd.sblk = f->d_sblk;
      cs.fd.sblk_page = f->d_sblk_page;
    cs.fd.sblk_ne = f->d_sblk + f->total_sblk;
      cs.scratch_base = P.s0;
      cs.open_sel = P.dict ? 1 : 2;
      OPEN_HIP(hipMemcpyAsync(d_cs, &cs, sizeof(cs), hipMemcpyHostToDevice, s));
      std::vector<Segment> segs{Segment{0, P.p0, P.p1, 0}};
      SegTable st2 = make_segs(segs);
      const uint32_t b0 = f->pages[P.p0].sblk_begin, b1 = P.p1 < npages ? f->pages[P.p1].sblk_begin : (uint32_t)sblk;
      if (b1 > b0) {
        std::vector<Segment> bsegs{Segment{0, b0, b1, 0}};
        hipLaunchKernelGGL(k_snappy_blk, dim3((b1 - b0 + 4 * SNAP_LANES - 1) / (4 * SNAP_LANES)), dim3(256), 0, s, d_cs,
                           make_segs(bsegs), (const uint32_t*)nullptr, 0u, d_scratch, f->d_err, 1);
      }
      hipLaunchKernelGGL(k_snappy, dim3(P.p1 - P.p0), dim3(64), 0, s, d_cs, st2, d_scratch, 1, f->d_err);
      if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_snappy launch failed"); }
    }
    // ---- DELTA_BYTE_ARRAY pages: facts, expansion layout, expansion ----
    if (!P.dict) {
      std::vector<ColScan> xc;
      std::vector<Segment> xs;
      uint32_t xw = 0;
      for (int c = 0; c < f->ncols; ++c) {
        if (f->cols[c].type != T_BYTE_ARRAY) continue;
        const uint32_t p0 = std::max(P.p0, f->chunk_page0[(size_t)c * f->nrg]),
                       p1 = std::min(P.p1, f->chunk_page0[(size_t)(c + 1) * f->nrg]);
        bool any = false;
        for (uint32_t pp = p0; pp < p1 && !any; ++pp) any = f->pages[pp].kind != PAGE_DICT && f->pages[pp].encoding == E_DBA;
        if (!any) continue;
        ColScan cs;
        memset(&cs, 0, sizeof(cs));
        cs.fd.file = file;
        cs.fd.pages = f->d_pages;
        cs.type = T_BYTE_ARRAY;
        cs.optional = f->cols[c].optional;
        cs.col = c;
        cs.page_begin = p0;
        cs.page_end = p1;
        xs.push_back(Segment{(uint32_t)xc.size(), p0, p1, xw});
        xw += p1 - p0;
        xc.push_back(cs);
      }
      const uint64_t xs0 = xscratch;
      for (uint32_t pp = P.p0; pp < P.p1; ++pp) f->xscratch_prefix[pp] = xscratch;
      if (!xc.empty()) {
        if (xs.size() > MAX_SEGS) { cleanup_open(); free_handle(f); return fail(PQ_EUNSUPPORTED, "too many DELTA_BYTE_ARRAY columns"); }
        if (hipMalloc(&d_xcols, sizeof(ColScan) * xc.size()) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: allocation failed"); }
        OPEN_HIP(hipMemcpyAsync(d_xcols, xc.data(), sizeof(ColScan) * xc.size(), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_dba, dim3(xw), dim3(64), 0, s, d_xcols, make_segs(xs), (uint8_t*)nullptr, scr,
                           (uint8_t*)nullptr, f->d_pages, 0, f->d_err);
        if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_dba launch failed"); }
        {
          pq_status stx = read_err(f, s);
          if (stx != PQ_OK) { cleanup_open(); free_handle(f); return stx; }
        }
        OPEN_HIP(hipMemcpy(f->pages.data() + P.p0, f->d_pages + P.p0, sizeof(PageDev) * (P.p1 - P.p0),
                           hipMemcpyDeviceToHost));
        for (uint32_t pp = P.p0; pp < P.p1; ++pp) {
          PageDev& pg = f->pages[pp];
          f->xscratch_prefix[pp] = xscratch;
          if (pg.kind == PAGE_DICT || pg.encoding != E_DBA || f->chunks[pg.chunk].type != T_BYTE_ARRAY ||
              pg.x_total == DBA_UNSUPPORTED)
            continue;
          pg.x_off = xscratch;
          xscratch += align_up((uint64_t)pg.xlen + SCRATCH_PAD, 16);
        }
        OPEN_HIP(hipMemcpyAsync(f->d_pages + P.p0, f->pages.data() + P.p0, sizeof(PageDev) * (P.p1 - P.p0),
                                hipMemcpyHostToDevice, s));
        if (xscratch > xs0) {
          if (hipMalloc(&d_xscratch_mem, OPEN_GUARD + (xscratch - xs0)) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: no device memory for expansion"); }
          d_xscratch = d_xscratch_mem + OPEN_GUARD;
          hipLaunchKernelGGL(k_dba, dim3(xw), dim3(64), 0, s, d_xcols, make_segs(xs), (uint8_t*)nullptr, scr,
                             d_xscratch - xs0, f->d_pages, 1, f->d_err);
          if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_dba launch failed"); }
          xscr = d_xscratch - xs0;
          xscr_lim = xscratch;
        }
      }
    }
    if (plist.empty()) {
      if (P.dict) {  // no dictionary pages: every chunk's slot says so
        pq_status st5 = build_dicts(f, scr, host_copy, s);
        if (st5 != PQ_OK) { cleanup_open(); free_handle(f); return st5; }
      }
      free_pass();
      continue;
    }
    // one wave per page, the longest walks first (string dictionaries by
    // bytes, then data pages by rows), so that they start at once instead of
    // behind the waves of earlier pages
    const uint32_t npl = (uint32_t)plist.size();
    std::vector<uint32_t> order(plist);
    std::vector<uint64_t> work(npages, 0);
    std::vector<uint32_t> lv_list;  // pages whose levels the k_lv kernels walk
    bool any_delta = false;         // pages that may have their blocks walked by the k_dl kernels
    bool any_dict = false;          // pages that may have their indices walked by the k_di kernels
    for (uint32_t p : plist) {
      const PageDev& pg = f->pages[p];
      const bool sdict = pg.kind == PAGE_DICT && f->chunks[pg.chunk].type == T_BYTE_ARRAY && pg.uncomp_size <= SCHAIN_MIN;
      work[p] = sdict ? 16ull * pg.uncomp_size : (uint64_t)(pg.num_values > 0 ? pg.num_values : 0);
      if (pg.kind != PAGE_DICT && lv_page(pg, f->chunks[pg.chunk].optional != 0)) lv_list.push_back(p);
      if (pg.kind != PAGE_DICT && (pg.encoding == E_DELTA || pg.encoding == E_DLBA)) any_delta = true;
      if (pg.kind != PAGE_DICT && (pg.encoding == E_PLAIN_DICT || pg.encoding == E_RLE_DICT)) any_dict = true;
    }
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return work[a] > work[b]; });
    if (hipMalloc(&d_order, sizeof(uint32_t) * npl) != hipSuccess ||
        hipMemcpy(d_order, order.data(), sizeof(uint32_t) * npl, hipMemcpyHostToDevice) != hipSuccess) {
      cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: page order");
    }
    hipLaunchKernelGGL(k_index, dim3(npl), dim3(64), 0, s, file, scr, f->d_pages, (int)npl, f->d_chunks, f->d_tiles,
                       f->d_strck, f->d_ckl, f->d_ckv, f->d_err, flim, scr_lim, d_order, xscr, xscr_lim, 1);
    if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_index launch failed"); }
    // long level streams: their exact lengths (stored by the launch above),
    // then candidates, link, tile entries, checkpoints and the value streams
    if (!lv_list.empty() || any_delta || any_dict) {
      OPEN_HIP(hipMemcpyAsync(f->pages.data() + P.p0, f->d_pages + P.p0, sizeof(PageDev) * (P.p1 - P.p0),
                              hipMemcpyDeviceToHost, s));
      OPEN_HIP(hipStreamSynchronize(s));
    }
    if (!lv_list.empty()) {
      std::vector<LvPage> lps;
      std::vector<uint32_t> seg_page, order2;
      for (uint32_t p : lv_list) {
        const PageDev& pg = f->pages[p];
        LvPage x;
        x.page = p;
        x.seg0 = (uint32_t)seg_page.size();
        x.nseg = (uint32_t)(((uint64_t)(pg.def_len > 0 ? pg.def_len : 0) + LV_SEG - 1) / LV_SEG);
        for (uint32_t j = 0; j < x.nseg; ++j) seg_page.push_back((uint32_t)lps.size());
        lps.push_back(x);
        order2.push_back(p);
      }
      std::stable_sort(order2.begin(), order2.end(), [&](uint32_t a, uint32_t b) { return work[a] > work[b]; });
      const size_t npg = lps.size(), nseg = seg_page.size();
      const size_t o_seg = align_up(sizeof(LvPage) * npg, 256), o_ord = align_up(o_seg + 4 * nseg, 256),
                   o_cand = align_up(o_ord + 4 * npg, 256),
                   o_ent = align_up(o_cand + sizeof(LvCand) * LV_CAND * nseg, 256),
                   o_ok = align_up(o_ent + sizeof(LvEntry) * nseg, 256), total = o_ok + 4 * npg;
      if (hipMalloc(&d_lv, total) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: level walk tables"); }
      LvPage* d_lps = reinterpret_cast<LvPage*>(d_lv);
      uint32_t* d_segp = reinterpret_cast<uint32_t*>(d_lv + o_seg);
      uint32_t* d_ord2 = reinterpret_cast<uint32_t*>(d_lv + o_ord);
      LvCand* d_cand = reinterpret_cast<LvCand*>(d_lv + o_cand);
      LvEntry* d_ent = reinterpret_cast<LvEntry*>(d_lv + o_ent);
      uint32_t* d_ok = reinterpret_cast<uint32_t*>(d_lv + o_ok);
      OPEN_HIP(hipMemcpyAsync(d_lps, lps.data(), sizeof(LvPage) * npg, hipMemcpyHostToDevice, s));
      if (nseg) OPEN_HIP(hipMemcpyAsync(d_segp, seg_page.data(), 4 * nseg, hipMemcpyHostToDevice, s));
      OPEN_HIP(hipMemcpyAsync(d_ord2, order2.data(), 4 * npg, hipMemcpyHostToDevice, s));
      if (nseg)
        hipLaunchKernelGGL(k_lv_cand, dim3((uint32_t)nseg), dim3(LV_CAND), 0, s, d_lps, d_segp, f->d_pages, file,
                           scr, flim, scr_lim, d_cand);
      hipLaunchKernelGGL(k_lv_link, dim3((uint32_t)((npg + 63) / 64)), dim3(64), 0, s, d_lps, (int)npg, f->d_pages,
                         d_cand, d_ent, d_ok, f->d_err);
      if (nseg)
        hipLaunchKernelGGL(k_lv_tiles, dim3((uint32_t)nseg), dim3(64), 0, s, d_lps, d_segp, d_ent, d_ok, f->d_pages,
                           file, scr, flim, scr_lim, f->d_tiles, f->d_ckl, f->d_err, 0);
      hipLaunchKernelGGL(k_lv_tiles, dim3((uint32_t)npg), dim3(64), 0, s, d_lps, d_segp, d_ent, d_ok, f->d_pages, file,
                         scr, flim, scr_lim, f->d_tiles, f->d_ckl, f->d_err, 1);
      hipLaunchKernelGGL(k_index, dim3((uint32_t)npg), dim3(64), 0, s, file, scr, f->d_pages, (int)npg,
                         f->d_chunks, f->d_tiles, f->d_strck, f->d_ckl, f->d_ckv, f->d_err, flim, scr_lim,
                         d_ord2, xscr, xscr_lim, 2);
      if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_lv launch failed"); }
    }
    // long DELTA block chains (headers parsed by the index pass above): block
    // positions, then every tile's entry block and checkpoints
    if (any_delta) {
      std::vector<DlPage> dps;
      std::vector<uint32_t> seg_page, tile_dp;
      uint64_t nblk = 0;
      for (uint32_t p : plist) {
        const PageDev& pg = f->pages[p];
        if (!dl_page(pg, f->chunks[pg.chunk].type)) continue;
        DlPage x;
        x.page = p;
        x.seg0 = (uint32_t)seg_page.size();
        x.nseg = (uint32_t)(((uint64_t)pg.val_len + DL_SEG - 1) / DL_SEG);
        x.blk0 = (uint32_t)nblk;
        x.tl0 = (uint32_t)tile_dp.size();
        x.maxw = f->chunks[pg.chunk].type == T_INT64 ? 64 : 32;
        nblk += ((uint64_t)pg.num_values + 127) / 128 + 1;  // blocks hold 128 values or more
        const uint32_t nt = (uint32_t)(((uint64_t)pg.num_values + TILE_ROWS - 1) / TILE_ROWS);
        for (uint32_t j = 0; j < x.nseg; ++j) seg_page.push_back((uint32_t)dps.size());
        for (uint32_t j = 0; j < nt; ++j) tile_dp.push_back((uint32_t)dps.size());
        dps.push_back(x);
      }
      if (nblk > 0xffffffffull) { cleanup_open(); free_handle(f); return fail(PQ_EUNSUPPORTED, "too many DELTA blocks"); }
      if (!dps.empty()) {
        const size_t npg = dps.size(), nseg = seg_page.size(), ntl = tile_dp.size();
        const size_t o_seg = align_up(sizeof(DlPage) * npg, 256), o_tl = align_up(o_seg + 4 * nseg, 256),
                     o_cand = align_up(o_tl + 4 * ntl, 256),
                     o_ent = align_up(o_cand + sizeof(DlCand) * DL_CAND * nseg, 256),
                     o_ok = align_up(o_ent + sizeof(DlEntry) * nseg, 256), o_blk = align_up(o_ok + 4 * npg, 256),
                     total = o_blk + 4 * (size_t)nblk;
        if (hipMalloc(&d_dl, total) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: DELTA walk tables"); }
        DlPage* d_dps = reinterpret_cast<DlPage*>(d_dl);
        uint32_t* d_segp = reinterpret_cast<uint32_t*>(d_dl + o_seg);
        uint32_t* d_tlp = reinterpret_cast<uint32_t*>(d_dl + o_tl);
        DlCand* d_cand = reinterpret_cast<DlCand*>(d_dl + o_cand);
        DlEntry* d_ent = reinterpret_cast<DlEntry*>(d_dl + o_ent);
        uint32_t* d_ok = reinterpret_cast<uint32_t*>(d_dl + o_ok);
        uint32_t* d_blk = reinterpret_cast<uint32_t*>(d_dl + o_blk);
        OPEN_HIP(hipMemcpyAsync(d_dps, dps.data(), sizeof(DlPage) * npg, hipMemcpyHostToDevice, s));
        if (nseg) OPEN_HIP(hipMemcpyAsync(d_segp, seg_page.data(), 4 * nseg, hipMemcpyHostToDevice, s));
        if (ntl) OPEN_HIP(hipMemcpyAsync(d_tlp, tile_dp.data(), 4 * ntl, hipMemcpyHostToDevice, s));
        if (nseg)
          hipLaunchKernelGGL(k_dl_cand, dim3((uint32_t)nseg), dim3(DL_CAND), 0, s, d_dps, d_segp, f->d_pages, file,
                             scr, flim, scr_lim, d_cand, f->d_err);
        hipLaunchKernelGGL(k_dl_link, dim3((uint32_t)((npg + 63) / 64)), dim3(64), 0, s, d_dps, (int)npg, f->d_pages,
                           d_cand, d_ent, d_ok, f->d_err);
        if (nseg)
          hipLaunchKernelGGL(k_dl_fill, dim3((uint32_t)nseg), dim3(64), 0, s, d_dps, d_segp, d_ent, d_ok, f->d_pages,
                             file, scr, flim, scr_lim, d_blk, f->d_err, 0);
        hipLaunchKernelGGL(k_dl_fill, dim3((uint32_t)npg), dim3(64), 0, s, d_dps, d_segp, d_ent, d_ok, f->d_pages,
                           file, scr, flim, scr_lim, d_blk, f->d_err, 1);
        if (ntl)
          hipLaunchKernelGGL(k_dl_tiles, dim3((uint32_t)((ntl + 255) / 256)), dim3(256), 0, s, d_dps, d_tlp, (int)ntl,
                             f->d_pages, f->d_tiles, f->d_ckv, d_blk, f->d_err);
        if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_dl launch failed"); }
      }
    }
    // long dictionary-index streams (widths parsed by the index pass above):
    // every tile's entry run and value checkpoints
    if (any_dict) {
      std::vector<DiPage> dps;
      std::vector<uint32_t> seg_page, tile_dp;
      for (uint32_t p : plist) {
        const PageDev& pg = f->pages[p];
        if (!di_page(pg)) continue;
        DiPage x;
        x.page = p;
        x.seg0 = (uint32_t)seg_page.size();
        x.nseg = (uint32_t)(((uint64_t)pg.val_len + DI_SEG - 1) / DI_SEG);
        x.tl0 = (uint32_t)tile_dp.size();
        const uint32_t nt = (uint32_t)(((uint64_t)pg.num_values + TILE_ROWS - 1) / TILE_ROWS);
        for (uint32_t j = 0; j < x.nseg; ++j) seg_page.push_back((uint32_t)dps.size());
        for (uint32_t j = 0; j < nt; ++j) tile_dp.push_back((uint32_t)dps.size());
        dps.push_back(x);
      }
      if (!dps.empty()) {
        const size_t npg = dps.size(), nseg = seg_page.size(), ntl = tile_dp.size();
        const size_t o_seg = align_up(sizeof(DiPage) * npg, 256), o_tl = align_up(o_seg + 4 * nseg, 256),
                     o_cand = align_up(o_tl + 4 * ntl, 256),
                     o_ent = align_up(o_cand + sizeof(DiCand) * DI_CAND_MAX * nseg, 256),
                     o_ok = align_up(o_ent + sizeof(DlEntry) * nseg, 256), total = o_ok + 4 * npg;
        if (hipMalloc(&d_di, total) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: index walk tables"); }
        DiPage* d_dps = reinterpret_cast<DiPage*>(d_di);
        uint32_t* d_segp = reinterpret_cast<uint32_t*>(d_di + o_seg);
        uint32_t* d_tlp = reinterpret_cast<uint32_t*>(d_di + o_tl);
        DiCand* d_cand = reinterpret_cast<DiCand*>(d_di + o_cand);
        DlEntry* d_ent = reinterpret_cast<DlEntry*>(d_di + o_ent);
        uint32_t* d_ok = reinterpret_cast<uint32_t*>(d_di + o_ok);
        OPEN_HIP(hipMemcpyAsync(d_dps, dps.data(), sizeof(DiPage) * npg, hipMemcpyHostToDevice, s));
        if (nseg) OPEN_HIP(hipMemcpyAsync(d_segp, seg_page.data(), 4 * nseg, hipMemcpyHostToDevice, s));
        if (ntl) OPEN_HIP(hipMemcpyAsync(d_tlp, tile_dp.data(), 4 * ntl, hipMemcpyHostToDevice, s));
        if (nseg)
          hipLaunchKernelGGL(k_di_cand, dim3((uint32_t)nseg), dim3(256), 0, s, d_dps, d_segp, f->d_pages, file,
                             scr, flim, scr_lim, d_cand, f->d_err);
        hipLaunchKernelGGL(k_di_link, dim3((uint32_t)((npg + 63) / 64)), dim3(64), 0, s, d_dps, (int)npg, f->d_pages,
                           d_cand, d_ent, d_ok, f->d_err);
        if (nseg)
          hipLaunchKernelGGL(k_di_fill, dim3((uint32_t)nseg), dim3(64), 0, s, d_dps, d_segp, d_ent, d_ok, f->d_pages,
                             file, scr, flim, scr_lim, f->d_tiles, f->d_err, 0);
        hipLaunchKernelGGL(k_di_fill, dim3((uint32_t)npg), dim3(64), 0, s, d_dps, d_segp, d_ent, d_ok, f->d_pages,
                           file, scr, flim, scr_lim, f->d_tiles, f->d_err, 1);
        if (ntl)
          hipLaunchKernelGGL(k_di_ckpt, dim3((uint32_t)((ntl + 3) / 4)), dim3(64), 0, s, d_dps, d_tlp, (int)ntl,
                             f->d_pages, f->d_tiles, file, scr, flim, scr_lim, f->d_ckv, f->d_err);
        if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_di launch failed"); }
      }
    }
    // long string dictionaries: their length chains, segments side by side
    std::vector<SChainPage> scp;
    std::vector<uint32_t> seg_page;
    for (uint32_t p : plist) {
      const PageDev& pg = f->pages[p];
      if (pg.kind != PAGE_DICT || f->chunks[pg.chunk].type != T_BYTE_ARRAY || pg.uncomp_size <= SCHAIN_MIN) continue;
      const bool in_scratch = pg.scratch_len > 0;
      SChainPage x;
      x.base = in_scratch ? scr : file;
      x.off = in_scratch ? pg.scratch_off : pg.payload;
      x.lim = in_scratch ? scr_lim : flim;
      x.len = (uint32_t)pg.uncomp_size;
      x.n = pg.num_values > 0 ? (uint32_t)pg.num_values : 0u;
      x.page = p;
      x.seg0 = (uint32_t)seg_page.size();
      x.nseg = (uint32_t)(((uint64_t)x.len + SCHAIN_SEG - 1) / SCHAIN_SEG);
      x.strck_begin = pg.strck_begin;
      for (uint32_t j = 0; j < x.nseg; ++j) seg_page.push_back((uint32_t)scp.size());
      scp.push_back(x);
    }
    if (!scp.empty()) {
      const size_t npg = scp.size(), nseg = seg_page.size();
      const size_t o_seg = align_up(sizeof(SChainPage) * npg, 256), o_cand = align_up(o_seg + 4 * nseg, 256),
                   o_start = align_up(o_cand + sizeof(SChainCand) * SCHAIN_CAND * nseg, 256),
                   o_base = align_up(o_start + 4 * nseg, 256), o_ok = align_up(o_base + 4 * nseg, 256),
                   total = o_ok + 4 * npg;
      if (hipMalloc(&d_schain, total) != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_ENOMEM, "open: dictionary chain tables"); }
      SChainPage* d_pgs = reinterpret_cast<SChainPage*>(d_schain);
      uint32_t* d_segp = reinterpret_cast<uint32_t*>(d_schain + o_seg);
      SChainCand* d_cand = reinterpret_cast<SChainCand*>(d_schain + o_cand);
      uint32_t* d_start = reinterpret_cast<uint32_t*>(d_schain + o_start);
      uint32_t* d_base = reinterpret_cast<uint32_t*>(d_schain + o_base);
      uint32_t* d_ok = reinterpret_cast<uint32_t*>(d_schain + o_ok);
      OPEN_HIP(hipMemcpyAsync(d_pgs, scp.data(), sizeof(SChainPage) * npg, hipMemcpyHostToDevice, s));
      OPEN_HIP(hipMemcpyAsync(d_segp, seg_page.data(), 4 * nseg, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_schain_cand, dim3((uint32_t)nseg), dim3(64), 0, s, d_pgs, d_segp, d_cand);
      hipLaunchKernelGGL(k_schain_link, dim3((uint32_t)((npg + 63) / 64)), dim3(64), 0, s, d_pgs, (int)npg, d_cand, d_start,
                         d_base, d_ok);
      hipLaunchKernelGGL(k_schain_fill, dim3((uint32_t)nseg), dim3(64), 0, s, d_pgs, d_segp, d_start, d_base, d_ok,
                         f->d_strck, f->d_pages, f->d_err);
      hipLaunchKernelGGL(k_schain_seq, dim3((uint32_t)npg), dim3(64), 0, s, d_pgs, (int)npg, d_ok, f->d_strck, f->d_pages,
                         f->d_err);
      if (hipGetLastError() != hipSuccess) { cleanup_open(); free_handle(f); return fail(PQ_EHIP, "k_schain launch failed"); }
    }
    if (P.dict) {
      // resident dictionaries, while the window holds the decompressed pages
      {
        pq_status st3 = read_err(f, s);
        if (st3 != PQ_OK) { cleanup_open(); free_handle(f); return st3; }
      }
      OPEN_HIP(hipMemcpy(f->pages.data(), f->d_pages, sizeof(PageDev) * npages, hipMemcpyDeviceToHost));
      pq_status st5 = build_dicts(f, scr, host_copy, s);
      if (st5 != PQ_OK) { cleanup_open(); free_handle(f); return st5; }
    }
    {
      pq_status st6 = read_err(f, s);  // the pass is done: its tables may go
      if (st6 != PQ_OK) { cleanup_open(); free_handle(f); return st6; }
    }
    free_pass();
  }
  f->xscratch_prefix[npages] = xscratch;
  HIP_OR(hipEventRecord(e1, s));
  {
    pq_status st3 = read_err(f, s);
    if (st3 != PQ_OK) { cleanup_open(); free_handle(f); return st3; }
  }
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (npages) OPEN_HIP(hipMemcpy(f->pages.data(), f->d_pages, sizeof(PageDev) * npages, hipMemcpyDeviceToHost));
  f->fd.file = file;
  f->fd.pages = f->d_pages;
  f->fd.tiles = f->d_tiles;
  f->fd.ckl = f->d_ckl;
  f->fd.ckv = f->d_ckv;
  f->fd.strck = f->d_strck;
  f->fd.sblk = f->d_sblk;
  f->fd.sblk_page = f->d_sblk_page;
  f->fd.sblk_ne = f->d_sblk ? f->d_sblk + f->total_sblk : nullptr;
  f->fd.dicts = f->d_dicts;
  cleanup_open();

#undef OPEN_HIP
#undef OPEN_ERR

  // ---- tile prefix (per-tile DELTA sums and string byte counts) ----
  const auto tp0 = std::chrono::steady_clock::now();
  {
    pq_status st4 = build_tile_prefix(f, s);
    if (st4 != PQ_OK) { free_handle(f); return st4; }
  }
  const double prefix_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tp0).count();

  // ---- statistics ----
  pq_file_stats& S = f->stats;
  for (const PageDev& pg : f->pages) {
    if (pg.kind == PAGE_DICT) S.dict_pages++;
    else S.pages++;
    if (pg.scratch_len) S.compressed_pages++;
    S.encoded_bytes += pg.comp_size;
    S.uncompressed_bytes += pg.uncomp_size;
  }
  S.tiles = (int64_t)tiles;
  S.open_ms_device = ms + prefix_ms;
  f->device_bytes += 4 + sizeof(ChunkDev) * (uint64_t)nchunks + sizeof(PageDev) * (uint64_t)npages +
                     (sizeof(TileDev) + 4ull * NLCK + sizeof(Ck) * NSUB) * tiles + 4ull * strck +
                     12ull * sblk +  // Snappy block index: offset, element count, page
                     8ull * (tiles + 1) + sizeof(DictSlot) * (uint64_t)nchunks;
  S.device_bytes = f->device_bytes;
  (void)t0;
  *out = f;
  return PQ_OK;
}

extern "C" pq_status pq_open_device(const void* dev_buf, uint64_t len, pq_stream stream, pq_file* out) {
  return open_impl(dev_buf, len, stream, false, out);
}

extern "C" pq_status pq_open_host(const void* host_buf, uint64_t len, pq_stream stream, pq_file* out) {
  if (!out) return fail(PQ_EINVAL, "out is NULL");
  *out = nullptr;
  if (!host_buf) return fail(PQ_EINVAL, "host_buf is NULL");
  if (len < 12) return fail(PQ_ECORRUPT, "file shorter than 12 bytes");
  hipStream_t s = (hipStream_t)stream;
  // the open-time passes read the file on the device: a temporary copy,
  // freed when the index is built
  uint8_t* tmp = nullptr;
  if (hipMalloc(&tmp, (len + 15) / 16 * 16 + 16) != hipSuccess) return fail(PQ_ENOMEM, "open: no device memory for the file");
  pq_status st = PQ_OK;
  if (hipMemcpyAsync(tmp, host_buf, len, hipMemcpyHostToDevice, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    st = fail(PQ_EHIP, "open: copy of the host file");
  if (st == PQ_OK) st = open_impl(tmp, len, stream, true, out);
  if (st == PQ_OK) {
    (void)hipStreamSynchronize(s);
    pq_file f = *out;
    f->file = nullptr;
    f->fd.file = nullptr;
    f->host = static_cast<const uint8_t*>(host_buf);
  }
  (void)hipFree(tmp);
  return st;
}

extern "C" void pq_close(pq_file f) { free_handle(f); }

extern "C" pq_status pq_num_row_groups(pq_file f, int32_t* n) {
  if (!f || !n) return fail(PQ_EINVAL, "NULL argument");
  *n = f->nrg;
  return PQ_OK;
}
extern "C" pq_status pq_num_columns(pq_file f, int32_t* n) {
  if (!f || !n) return fail(PQ_EINVAL, "NULL argument");
  *n = f->ncols;
  return PQ_OK;
}
extern "C" pq_status pq_column_info_get(pq_file f, int32_t col, pq_column_info* out) {
  if (!f || !out || col < 0 || col >= f->ncols) return fail(PQ_EINVAL, "bad column");
  out->type = f->cols[col].type;
  out->nullable = f->cols[col].optional;
  memset(out->name, 0, sizeof(out->name));
  strncpy(out->name, f->cols[col].name.c_str(), sizeof(out->name) - 1);
  return PQ_OK;
}
extern "C" pq_status pq_row_group_rows(pq_file f, int32_t rg, int64_t* rows) {
  if (!f || !rows || rg < 0 || rg >= f->nrg) return fail(PQ_EINVAL, "bad row group");
  *rows = f->rg_rows[rg];
  return PQ_OK;
}
extern "C" pq_status pq_file_stats_get(pq_file f, pq_file_stats* out) {
  if (!f || !out) return fail(PQ_EINVAL, "NULL argument");
  *out = f->stats;
  return PQ_OK;
}

// ---------------------------------------------------------------------------
// resident dictionaries (built once, at open)
// ---------------------------------------------------------------------------
// Every dictionary page of the file becomes a DictSlot of its chunk: the
// fixed-width array (the page body itself when it is uncompressed and
// aligned, else a copy made by k_dict), or for strings the body (copied out
// of the decompression buffer when the page is compressed), (position,
// length) pairs, the length array and, for dictionaries that serve at least
// SLOT_ROWS_PER_ENTRY rows of their row group per entry, 64-byte slots.
// `scratch` holds the decompressed pages at their file-wide scratch offsets.
static pq_status build_dicts(pq_file f, const uint8_t* scratch, bool copy_all, hipStream_t s) {
  const int nchunks = f->ncols * f->nrg;
  f->dicts.assign((size_t)nchunks, DictSlot{});
  std::vector<DictWork> work;
  struct Copy { uint64_t dst; uint64_t src; uint64_t n; bool from_scratch; };
  std::vector<Copy> copies;  // decompressed string dictionary bodies -> arena
  uint64_t off = 0;
  uint32_t units = 0;
  for (int q = 0; q < nchunks; ++q) {
    DictSlot& sl = f->dicts[(size_t)q];
    memset(&sl, 0, sizeof(sl));
    sl.page = ~0u;
    sl.type = f->chunks[(size_t)q].type;
    const uint32_t p0 = f->chunk_page0[(size_t)q];
    if (p0 >= f->chunk_page0[(size_t)q + 1] || f->pages[p0].kind != PAGE_DICT) continue;
    const PageDev& pg = f->pages[p0];
    const bool comp = (pg.flags & 2) != 0;
    sl.page = p0;
    sl.n = (uint32_t)(pg.num_values > 0 ? pg.num_values : 0);
    const uint64_t n = sl.n;
    uint32_t nu = 0;
    if (sl.type != T_BYTE_ARRAY) {
      const uint64_t w = sl.type == T_INT32 ? 4 : 8;
      if (!comp && !copy_all && ((uintptr_t)(f->file + pg.val_off) % w) == 0) {
        sl.entries = const_cast<uint8_t*>(f->file + pg.val_off);  // the body is the array
        continue;
      }
      sl.body = comp ? scratch : f->file;
      sl.body_off = pg.val_off;
      sl.entries = reinterpret_cast<uint8_t*>(off);  // arena offset until the arena exists
      off = align_up(off + w * n + 16, 256);
      nu = (uint32_t)((n + DICT_FIXED_PER - 1) / DICT_FIXED_PER);
    } else {
      if (comp || copy_all) {
        sl.body = reinterpret_cast<const uint8_t*>(off);
        sl.body_off = 0;
        copies.push_back(Copy{off, pg.val_off, pg.val_len, comp});
        off = align_up(off + pg.val_len + SCRATCH_PAD, 256);
      } else {
        sl.body = f->file;
        sl.body_off = pg.val_off;
      }
      sl.entries = reinterpret_cast<uint8_t*>(off);
      off = align_up(off + 8 * n + 16, 256);
      if (pg.dict_maxlen < 65536) sl.flags |= DICT_LENS16;
      sl.lens = reinterpret_cast<uint8_t*>(off);
      off = align_up(off + ((sl.flags & DICT_LENS16) ? 2 : 4) * n + 16, 256);
      const int g = q % f->nrg;
      if (pg.dict_maxlen <= SLOT_CHARS && n * SLOT_BYTES < (1ull << 32) &&
          n * SLOT_ROWS_PER_ENTRY <= (uint64_t)f->rg_rows[(size_t)g]) {
        sl.flags |= DICT_SLOTS;
        sl.slots = reinterpret_cast<uint8_t*>(off);
        off = align_up(off + SLOT_BYTES * n, 256);
      }
      nu = (uint32_t)(((n + STR_CK - 1) / STR_CK + DICT_CK_PER - 1) / DICT_CK_PER);
    }
    if (nu) {
      work.push_back(DictWork{(uint32_t)q, nu, units, 0});
      units += nu;
    }
  }
  if (off) {
    if (hipMalloc(&f->d_dict_arena, off) != hipSuccess) return fail(PQ_ENOMEM, "open: no device memory for dictionaries");
    f->device_bytes += off;
  }
  auto rebase = [&](const uint8_t* x) { return f->d_dict_arena + reinterpret_cast<uintptr_t>(x); };
  for (int q = 0; q < nchunks; ++q) {
    DictSlot& sl = f->dicts[(size_t)q];
    if (sl.page == ~0u) continue;
    const PageDev& pg = f->pages[sl.page];
    const bool comp = (pg.flags & 2) != 0;
    if (sl.type != T_BYTE_ARRAY) {
      if (sl.body) sl.entries = rebase(sl.entries);
      continue;
    }
    if (comp || copy_all) sl.body = rebase(sl.body);
    sl.entries = rebase(sl.entries);
    sl.lens = rebase(sl.lens);
    if (sl.flags & DICT_SLOTS) sl.slots = rebase(sl.slots);
  }
  for (const Copy& c : copies)
    HIP_OR(hipMemcpyAsync(f->d_dict_arena + c.dst, (c.from_scratch ? scratch : f->file) + c.src, c.n,
                          hipMemcpyDeviceToDevice, s));
  HIP_OR(hipMalloc(&f->d_dicts, sizeof(DictSlot) * (size_t)(nchunks ? nchunks : 1)));
  if (nchunks)
    HIP_OR(hipMemcpyAsync(f->d_dicts, f->dicts.data(), sizeof(DictSlot) * (size_t)nchunks, hipMemcpyHostToDevice, s));
  if (units) {
    DictWork* d_work = nullptr;
    HIP_OR(hipMalloc(&d_work, sizeof(DictWork) * work.size()));
    hipError_t e = hipMemcpyAsync(d_work, work.data(), sizeof(DictWork) * work.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_dict, dim3((units + 3) / 4), dim3(256), 0, s, f->d_pages, f->d_strck, f->d_dicts, d_work,
                         (uint32_t)work.size(), f->d_err);
      e = hipGetLastError();
    }
    pq_status st = e == hipSuccess ? read_err(f, s) : fail(PQ_EHIP, "open: k_dict: %s", hipGetErrorString(e));
    (void)hipFree(d_work);
    if (st != PQ_OK) return st;
  }
  // fixed-width copies no longer need their source; the decompression buffer
  // is freed after the open
  bool changed = false;
  for (DictSlot& sl : f->dicts)
    if (sl.page != ~0u && sl.type != T_BYTE_ARRAY && sl.body) { sl.body = nullptr; sl.body_off = 0; changed = true; }
  if (changed)
    HIP_OR(hipMemcpyAsync(f->d_dicts, f->dicts.data(), sizeof(DictSlot) * (size_t)nchunks, hipMemcpyHostToDevice, s));
  HIP_OR(hipStreamSynchronize(s));
  return PQ_OK;
}

// ---------------------------------------------------------------------------
// scan planning
// ---------------------------------------------------------------------------
namespace {

// Workspace header: the scan's error word (first error wins; code | page << 8)
// in the first 256 bytes, then the column table and the string-column list.
constexpr uint64_t WS_HEADER = 256;

struct Plan {
  std::vector<ColScan> cols;
  int64_t rows = 0;
  uint64_t ws_cols = 0, ws_which = 0, ws_total = 0;
  // launch lists
  std::vector<Segment> snappy_segs, prep_segs, pre_segs, fixed_segs[8], delta_segs, str_segs[2], edge_segs;
  std::vector<int32_t> str_cols;    // string ColScan indices (k_str_total)
  // units: pages (k_snappy), tiles (k_prep threads; one wave per tile elsewhere)
  std::vector<Segment> sblk_segs;  // k_snappy_blk: blocks of the compressed pages, one lane each
  std::vector<Segment> dba_segs;   // k_dba: pages of columns with DELTA_BYTE_ARRAY pages, one wave each
  uint32_t dba_waves = 0;
  uint32_t sblk_lanes = 0;
  uint64_t ws_sord = 0;  // k_snap_order's density buckets (0: blocks taken in segment order)
  bool str_spread[2] = {false, false}, fixed_spread[8] = {};  // columns interleaved wave by wave
  uint32_t snappy_waves = 0, prep_threads = 0, pre_units = 0, fixed_units[8] = {}, delta_units = 0, str_units[2] = {0, 0},
           edge_threads = 0;
  // a host-resident file: two staging slots for row groups in flight and
  // one column table per row group (its file base in its slot)
  uint64_t ws_stage = 0, stage_bytes = 0, ws_rgcols = 0;
  std::vector<uint64_t> rg_lo;  // per scanned row group: the lowest file offset of its selected chunks
};

// Work lists and workspace layout of a scan of `mask` over row groups
// [rg_b, rg_e).  With `index`, the plan of the open-time prefix pass instead:
// decompression and k_prepass of the columns that need a tile prefix, with a
// per-tile array in the workspace.
// One selected column of a scan: its table entry (workspace offsets from
// `off` on) and which decoders its pages need.
struct ColSetup {
  ColScan cs;
  bool has_delta = false, has_plain = false, has_dict = false, has_slots = false, has_bss = false;
  uint32_t nt = 0;        // tiles
  uint64_t sbytes = 0;    // decompressed bytes of its compressed pages
  uint64_t xbytes = 0;    // expansion bytes of its DELTA_BYTE_ARRAY pages
  uint32_t b0 = 0, b1 = 0;  // its Snappy blocks
};

// pr0/pr1 (index plans only): the pages [pr0, pr1) of the chunks instead of
// all of them.
void col_setup(pq_file f, int c, int32_t rg_b, int32_t rg_e, int64_t rows, uint64_t& off, bool index, ColSetup& k,
               uint32_t pr0 = ~0u, uint32_t pr1 = ~0u) {
  ColScan& cs = k.cs;
  memset(&cs, 0, sizeof(cs));
  cs.fd = f->fd;
  cs.type = f->cols[c].type;
  cs.optional = f->cols[c].optional;
  cs.width = cs.type == T_INT32 ? 4 : (cs.type == T_BYTE_ARRAY ? 0 : 8);
  cs.col = c;
  const uint32_t q0 = (uint32_t)(c * f->nrg + rg_b), q1 = (uint32_t)(c * f->nrg + rg_e);
  cs.tile_begin = f->chunk_tile0[q0];
  cs.tile_end = f->chunk_tile0[q1];
  cs.page_begin = f->chunk_page0[q0];
  cs.page_end = f->chunk_page0[q1];
  cs.row_base = f->rg_row0[rg_b];
  cs.rows = rows;
  if (pr0 != ~0u) {
    cs.page_begin = pr0;
    cs.page_end = pr1;
    uint32_t tb = ~0u, te = 0;
    for (uint32_t p = pr0; p < pr1; ++p) {
      const PageDev& pg = f->pages[p];
      if (pg.kind == PAGE_DICT) continue;
      tb = std::min(tb, pg.tile_begin);
      te = std::max(te, pg.tile_begin + (uint32_t)(((uint64_t)pg.num_values + TILE_ROWS - 1) / TILE_ROWS));
    }
    cs.tile_begin = tb == ~0u ? te : tb;
    cs.tile_end = te;
  }
  cs.scratch_base = f->scratch_prefix[cs.page_begin];
  k.sbytes = f->scratch_prefix[cs.page_end] - cs.scratch_base;
  cs.ws_scratch = off;
  off = align_up(off + k.sbytes, 256);
  cs.xscratch_base = f->xscratch_prefix[cs.page_begin];
  k.xbytes = f->xscratch_prefix[cs.page_end] - cs.xscratch_base;
  cs.ws_xscratch = off;
  off = align_up(off + k.xbytes, 256);
  for (uint32_t p = cs.page_begin; p < cs.page_end; ++p) {
    if (f->pages[p].kind == PAGE_DICT) continue;
    const int e = f->pages[p].encoding;
    if (e == E_DELTA) {
      k.has_delta = true;
    } else if (e == E_BSS && cs.type != T_BYTE_ARRAY) {
      k.has_bss = true;
    } else if (e == E_PLAIN_DICT || e == E_RLE_DICT) {
      if (cs.type == T_BYTE_ARRAY && (f->dicts[f->pages[p].chunk].flags & DICT_SLOTS))
        k.has_slots = true;
      else
        k.has_dict = true;
    } else {
      k.has_plain = true;  // PLAIN, or an encoding the kernel reports as unsupported
    }
  }
  k.nt = cs.tile_end - cs.tile_begin;
  if (cs.optional && k.nt) {
    cs.ws_edge = off;
    off = align_up(off + 8ull * k.nt, 256);
  }
  if (index && (cs.type == T_BYTE_ARRAY || k.has_delta)) {
    cs.ws_tile_aux = off;
    off = align_up(off + 8ull * (k.nt + 1), 256);
  }
  if (k.sbytes) {
    k.b0 = f->pages[cs.page_begin].sblk_begin;
    k.b1 = cs.page_end < (uint32_t)f->pages.size() ? f->pages[cs.page_end].sblk_begin : (uint32_t)f->total_sblk;
  }
}

pq_status make_plan(pq_file f, uint64_t mask, int32_t rg_b, int32_t rg_e, Plan& P, bool index = false,
                    uint32_t pr0 = ~0u, uint32_t pr1 = ~0u) {
  if (rg_b < 0 || rg_e > f->nrg || rg_b > rg_e) return fail(PQ_EINVAL, "bad row-group range [%d, %d)", rg_b, rg_e);
  if (f->ncols < 64 && (mask >> f->ncols)) return fail(PQ_EINVAL, "column mask selects missing columns");
  P.rows = f->rg_row0[rg_e] - f->rg_row0[rg_b];
  int ncs = __builtin_popcountll(mask);
  P.ws_cols = WS_HEADER;
  uint64_t off = align_up(P.ws_cols + sizeof(ColScan) * (ncs ? ncs : 1), 256);
  P.ws_which = off;
  off = align_up(off + sizeof(int32_t) * 64, 256);
  for (int c = 0; c < f->ncols; ++c) {
    if (!((mask >> c) & 1)) continue;
    ColSetup k;
    col_setup(f, c, rg_b, rg_e, P.rows, off, index, k, pr0, pr1);
    const ColScan& cs = k.cs;
    const uint32_t nt = k.nt;
    const uint32_t idx = (uint32_t)P.cols.size();
    if (index && cs.ws_tile_aux && nt) {
      P.pre_segs.push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.pre_units});
      P.pre_units += nt;
    }
    if (nt) {
      if (cs.type == T_BYTE_ARRAY) {
        for (int kk = 0; kk < 2; ++kk) {  // k_decode_str<kk>: tiles of slot dictionaries (1) or the others (0)
          if (!(kk ? k.has_slots : (k.has_plain || k.has_dict || k.has_delta))) continue;
          P.str_segs[kk].push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.str_units[kk]});
          P.str_units[kk] += nt;
        }
      } else {
        if (k.has_delta) {
          P.delta_segs.push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.delta_units});
          P.delta_units += nt;
        }
        const int wide = cs.width == 8 ? FX_WIDE : 0;
        for (int kind : {0, (int)FX_DICT, (int)FX_BSS}) {
          if (!(kind == FX_DICT ? k.has_dict : kind == FX_BSS ? k.has_bss : k.has_plain)) continue;
          const int K = kind | wide;
          P.fixed_segs[K].push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.fixed_units[K]});
          P.fixed_units[K] += nt;
        }
      }
      if (!cs.optional) {
        P.prep_segs.push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.prep_threads});
        P.prep_threads += nt;
      } else {
        P.edge_segs.push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.edge_threads});
        P.edge_threads += nt;
      }
    }
    if (cs.type == T_BYTE_ARRAY) P.str_cols.push_back((int32_t)idx);
    if (k.sbytes) {
      P.snappy_segs.push_back(Segment{idx, cs.page_begin, cs.page_end, P.snappy_waves});
      P.snappy_waves += cs.page_end - cs.page_begin;
      if (k.b1 > k.b0) {
        P.sblk_segs.push_back(Segment{idx, k.b0, k.b1, P.sblk_lanes});
        P.sblk_lanes += k.b1 - k.b0;
      }
    }
    if (k.xbytes) {
      P.dba_segs.push_back(Segment{idx, cs.page_begin, cs.page_end, P.dba_waves});
      P.dba_waves += cs.page_end - cs.page_begin;
    }
    P.cols.push_back(cs);
  }
  // The string kernel's columns, and those of the 8-byte dictionary kernel,
  // run side by side: wave u takes tile u / n of column u % n (a 10^6-entry
  // dictionary bound by random gathers beside small ones bound by instruction
  // issue).  Interleaving the other fixed-width kinds made them 1-3 % slower
  // (streaming columns gain nothing from the mix), so they stay in order.
  if (P.fixed_segs[FX_WIDE | FX_DICT].size() >= 2) {
    const int K = FX_WIDE | FX_DICT;
    uint32_t most = 0;
    for (const Segment& sg : P.fixed_segs[K]) most = std::max(most, sg.t1 - sg.t0);
    P.fixed_spread[K] = true;
    P.fixed_units[K] = (uint32_t)P.fixed_segs[K].size() * most;
  }
  for (int k = 0; k < 2; ++k) {
    if (P.str_segs[k].size() < 2) continue;
    uint32_t most = 0;
    for (const Segment& sg : P.str_segs[k]) most = std::max(most, sg.t1 - sg.t0);
    P.str_spread[k] = true;
    P.str_units[k] = (uint32_t)P.str_segs[k].size() * most;
  }
  if (!index && P.sblk_lanes && f->total_sblk < (1ull << SNAP_ORD_BITS) && P.cols.size() <= 64) {
    P.ws_sord = off;  // SNAP_BUCKETS counters, then SNAP_BUCKETS lists of sblk_lanes entries
    off = align_up(off + 256 + sizeof(uint32_t) * SNAP_BUCKETS * (uint64_t)P.sblk_lanes, 256);
  }
  if (f->host && !index && !P.cols.empty()) {
    uint64_t most = 0;
    for (int g = rg_b; g < rg_e; ++g) {
      uint64_t lo = ~0ull, hi = 0;
      for (const ColScan& cs : P.cols) {
        const ChunkDev& ch = f->chunks[(size_t)cs.col * f->nrg + g];
        lo = std::min(lo, ch.start);
        hi = std::max(hi, ch.end);
      }
      P.rg_lo.push_back(lo);
      most = std::max(most, hi - lo);
    }
    P.stage_bytes = align_up(most + 64, 256);  // reads may run 16 bytes past a stream
    P.ws_stage = off;
    off += 2 * P.stage_bytes;
    P.ws_rgcols = off;
    off = align_up(off + sizeof(ColScan) * P.cols.size() * (size_t)(rg_e - rg_b), 256);
  }
  P.ws_total = std::max<uint64_t>(off, 256);
  return PQ_OK;
}

}  // namespace

using FixedKernel = void (*)(uint8_t*, const ColScan*, SegTable, uint32_t*);
// The k_decode_fixed instantiation for kind K (FX_DICT | FX_WIDE | FX_BSS bits).
static FixedKernel fixed_kernel(int K) {
  switch (K) {
    case 0: return k_decode_fixed<0>;
    case FX_DICT: return k_decode_fixed<FX_DICT>;
    case FX_WIDE: return k_decode_fixed<FX_WIDE>;
    case FX_DICT | FX_WIDE: return k_decode_fixed<FX_DICT | FX_WIDE>;
    case FX_BSS: return k_decode_fixed<FX_BSS>;
    default: return k_decode_fixed<FX_BSS | FX_WIDE>;
  }
}

// The workspace header of a plan: the cleared error word, the column table
// and the string-column list, in one host-to-device copy.
static pq_status upload_header(Plan& P, uint8_t* ws, hipStream_t s) {
  std::vector<uint8_t> hdr(P.ws_which + sizeof(int32_t) * P.str_cols.size(), 0);
  if (!P.cols.empty()) memcpy(hdr.data() + P.ws_cols, P.cols.data(), sizeof(ColScan) * P.cols.size());
  if (!P.str_cols.empty()) memcpy(hdr.data() + P.ws_which, P.str_cols.data(), sizeof(int32_t) * P.str_cols.size());
  HIP_OR(hipMemcpyAsync(ws, hdr.data(), hdr.size(), hipMemcpyHostToDevice, s));
  return PQ_OK;
}

// Snappy decompression of the plan's compressed data pages (column table
// d_cols).
// sord_off, sord_cap: the workspace region of k_snap_order's buckets and
// their capacity (a plan's ws_sord and sblk_lanes; 0: segment order).
static pq_status enqueue_decompress(pq_file f, const Plan& P, const ColScan* d_cols, uint8_t* ws, uint32_t* err,
                                    hipStream_t s, uint64_t sord_off, uint32_t sord_cap) {
  for (const auto* v : {&P.snappy_segs, &P.sblk_segs, &P.dba_segs, &P.prep_segs, &P.pre_segs, &P.fixed_segs[0], &P.fixed_segs[1], &P.fixed_segs[2],
                        &P.fixed_segs[3], &P.fixed_segs[4], &P.fixed_segs[6], &P.delta_segs, &P.str_segs[0], &P.str_segs[1],
                        &P.edge_segs})
    if (v->size() > MAX_SEGS) return fail(PQ_EUNSUPPORTED, "too many segments");
  if (P.snappy_waves) {
    ProfScope ps_(f, KP_SNAPPY, s);
    hipLaunchKernelGGL(k_snappy, dim3(P.snappy_waves), dim3(64), 0, s, d_cols, make_segs(P.snappy_segs), ws, 0, err);
    HIP_OR(hipGetLastError());
  }
  if (P.sblk_lanes) {
    ProfScope ps_(f, KP_SNAPPY_BLK, s);
    uint32_t* sord = nullptr;
    if (sord_off && sord_cap >= P.sblk_lanes) {  // the blocks in buckets of density, the densest first
      sord = (uint32_t*)(ws + sord_off);
      hipLaunchKernelGGL(k_snap_order, dim3(1), dim3(256), 0, s, d_cols, make_segs(P.sblk_segs), ws, sord,
                         sord_cap, 0);
      hipLaunchKernelGGL(k_snap_order, dim3((P.sblk_lanes + 255) / 256), dim3(256), 0, s, d_cols,
                         make_segs(P.sblk_segs), ws, sord, sord_cap, 1);
      HIP_OR(hipGetLastError());
    }
    hipLaunchKernelGGL(k_snappy_blk, dim3((P.sblk_lanes + 4 * SNAP_LANES - 1) / (4 * SNAP_LANES)), dim3(256), 0, s,
                       d_cols, make_segs(P.sblk_segs), (const uint32_t*)sord, sord_cap, ws, err, 0);
    HIP_OR(hipGetLastError());
  }
  if (P.dba_waves) {  // DELTA_BYTE_ARRAY pages (after their decompression) to the PLAIN layout
    hipLaunchKernelGGL(k_dba, dim3(P.dba_waves), dim3(64), 0, s, d_cols, make_segs(P.dba_segs), ws,
                       (const uint8_t*)nullptr, (uint8_t*)nullptr, (PageDev*)nullptr, 1, err);
    HIP_OR(hipGetLastError());
  }
  return PQ_OK;
}

// Decompression and the upload: the steps the open-time prefix pass and a
// scan share.
static pq_status enqueue_front(pq_file f, Plan& P, uint8_t* ws, uint32_t* err, hipStream_t s) {
  pq_status st = upload_header(P, ws, s);
  if (st != PQ_OK) return st;
  return enqueue_decompress(f, P, reinterpret_cast<ColScan*>(ws + P.ws_cols), ws, err, s, P.ws_sord, P.sblk_lanes);
}

// The open-time prefix pass of a plan made with index = true: per-tile DELTA
// sums and string byte counts into the workspace's tile arrays (mode 1: the
// DELTA sums of DELTA_LENGTH_BYTE_ARRAY length streams only).
static pq_status enqueue_index(pq_file f, Plan& P, uint8_t* ws, int mode, hipStream_t s) {
  pq_status st = enqueue_front(f, P, ws, f->d_err, s);
  if (st != PQ_OK) return st;
  if (P.pre_units) {
    hipLaunchKernelGGL(k_prepass, dim3((P.pre_units + 3) / 4), dim3(256), 0, s, ws,
                       reinterpret_cast<ColScan*>(ws + P.ws_cols), make_segs(P.pre_segs), mode, f->d_err);
    HIP_OR(hipGetLastError());
  }
  return PQ_OK;
}

// REQUIRED validity and the decode kernels of a plan's tiles (column table
// d_cols), one launch per kernel kind.
static pq_status enqueue_decode(pq_file f, const Plan& P, const ColScan* d_cols, uint8_t* ws, uint32_t* err,
                                hipStream_t s) {
  if (P.prep_threads) {
    ProfScope ps_(f, KP_PREP, s);
    hipLaunchKernelGGL(k_prep, dim3((P.prep_threads + 255) / 256), dim3(256), 0, s, d_cols, make_segs(P.prep_segs));
    HIP_OR(hipGetLastError());
  }
  for (int K = 0; K < 8; ++K) {
    if (!P.fixed_units[K]) continue;
    ProfScope ps_(f, KP_FIXED0 + K, s);
    auto kern = fixed_kernel(K);
    hipLaunchKernelGGL(kern, dim3((P.fixed_units[K] + 3) / 4), dim3(256), 0, s, ws, d_cols,
                       make_segs(P.fixed_segs[K], P.fixed_spread[K]), err);
    HIP_OR(hipGetLastError());
  }
  if (P.delta_units) {
    ProfScope ps_(f, KP_DELTA, s);
    hipLaunchKernelGGL(k_decode_delta, dim3((P.delta_units + 3) / 4), dim3(256), 0, s, ws, d_cols,
                       make_segs(P.delta_segs), err);
    HIP_OR(hipGetLastError());
  }
  for (int k = 0; k < 2; ++k) {
    if (!P.str_units[k]) continue;
    ProfScope ps_(f, k ? KP_STR_SLOTS : KP_STR, s);
    hipLaunchKernelGGL(k ? k_decode_str<true> : k_decode_str<false>, dim3((P.str_units[k] + 3) / 4), dim3(256), 0, s,
                       ws, d_cols, make_segs(P.str_segs[k], P.str_spread[k]), err);
    HIP_OR(hipGetLastError());
  }
  return PQ_OK;
}

// offsets[rows] of string columns and the validity words tiles share.
static pq_status enqueue_finish(pq_file f, const Plan& P, const ColScan* d_cols, uint8_t* ws, uint32_t* err,
                                hipStream_t s) {
  if (!P.str_cols.empty()) {
    ProfScope ps_(f, KP_STR_TOTAL, s);
    hipLaunchKernelGGL(k_str_total, dim3(((uint32_t)P.str_cols.size() + 63) / 64), dim3(64), 0, s, d_cols,
                       reinterpret_cast<const int32_t*>(ws + P.ws_which), (int32_t)P.str_cols.size(), err);
    HIP_OR(hipGetLastError());
  }
  if (P.edge_threads) {
    ProfScope ps_(f, KP_EDGES, s);
    hipLaunchKernelGGL(k_edges, dim3((P.edge_threads + 255) / 256), dim3(256), 0, s, ws, d_cols, make_segs(P.edge_segs));
    HIP_OR(hipGetLastError());
  }
  return PQ_OK;
}

static pq_status enqueue(pq_file f, Plan& P, uint8_t* ws, hipStream_t s) {
  uint32_t* err = reinterpret_cast<uint32_t*>(ws);  // the scan's error word
  pq_status st = enqueue_front(f, P, ws, err, s);
  if (st != PQ_OK) return st;
  const ColScan* d_cols = reinterpret_cast<const ColScan*>(ws + P.ws_cols);
  // the string totals first (they read only the tile prefix), then the
  // decode kernels, then the shared validity words
  if (!P.str_cols.empty()) {
    ProfScope ps_(f, KP_STR_TOTAL, s);
    hipLaunchKernelGGL(k_str_total, dim3(((uint32_t)P.str_cols.size() + 63) / 64), dim3(64), 0, s, d_cols,
                       reinterpret_cast<const int32_t*>(ws + P.ws_which), (int32_t)P.str_cols.size(), err);
    HIP_OR(hipGetLastError());
  }
  st = enqueue_decode(f, P, d_cols, ws, err, s);
  if (st != PQ_OK) return st;
  if (P.edge_threads) {
    ProfScope ps_(f, KP_EDGES, s);
    hipLaunchKernelGGL(k_edges, dim3((P.edge_threads + 255) / 256), dim3(256), 0, s, ws, d_cols, make_segs(P.edge_segs));
    HIP_OR(hipGetLastError());
  }
  return PQ_OK;
}

// Builds the tile prefix at open: for every column with string or DELTA
// pages, the prefix pass over its row groups (in batches whose workspace
// stays below INDEX_WS_CAP), then the prefix sum on the host.
constexpr uint64_t INDEX_WS_CAP = 512ull << 20;

// One prefix pass (k_prepass in `mode`) over the tiles of every column that
// `need` selects, in row-group batches; fills val[t] for their tiles.
// One index plan over columns `mask` and row groups [g0, g0 + n): its
// per-tile values into val.
static pq_status prefix_plan(pq_file f, int mode, Plan& P, std::vector<uint64_t>& val, hipStream_t s) {
  if (!P.pre_units) return PQ_OK;
  uint8_t* ws = nullptr;
  if (hipMalloc(&ws, P.ws_total) != hipSuccess) return fail(PQ_ENOMEM, "open: no device memory for the prefix pass");
  pq_status st = enqueue_index(f, P, ws, mode, s);
  for (const ColScan& cs : P.cols) {
    const uint32_t cnt = cs.tile_end - cs.tile_begin;
    if (st == PQ_OK && cs.ws_tile_aux && cnt &&
        hipMemcpyAsync(val.data() + cs.tile_begin, ws + cs.ws_tile_aux, 8ull * cnt, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
      st = fail(PQ_EHIP, "open: prefix pass copy");
  }
  if (st == PQ_OK) st = read_err(f, s);
  (void)hipStreamSynchronize(s);
  (void)hipFree(ws);
  return st;
}

static pq_status prefix_pass(pq_file f, int mode, const std::vector<bool>& need, std::vector<uint64_t>& val,
                             hipStream_t s) {
  // every needed column at once (one decompression and one prepass launch
  // per batch of row groups), the batches sized to INDEX_WS_CAP; a single
  // row group over the cap is taken one column at a time
  uint64_t mask = 0;
  for (int c = 0; c < f->ncols; ++c)
    if (need[(size_t)c]) mask |= 1ull << c;
  if (!mask) return PQ_OK;
  for (int g0 = 0; g0 < f->nrg;) {
    int n = f->nrg - g0;
    Plan P;
    for (;;) {
      P = Plan();
      pq_status st = make_plan(f, mask, g0, g0 + n, P, true);
      if (st != PQ_OK) return st;
      if (P.ws_total <= INDEX_WS_CAP || n == 1) break;
      n = (n + 1) / 2;
    }
    if (P.ws_total <= INDEX_WS_CAP || __builtin_popcountll(mask) == 1) {
      pq_status st = prefix_plan(f, mode, P, val, s);
      if (st != PQ_OK) return st;
    } else {
      // one column at a time, and a column over the cap in runs of pages
      for (int c = 0; c < f->ncols; ++c) {
        if (!((mask >> c) & 1)) continue;
        Plan Q;
        pq_status st = make_plan(f, 1ull << c, g0, g0 + n, Q, true);
        if (st != PQ_OK) return st;
        if (Q.ws_total <= INDEX_WS_CAP) {
          st = prefix_plan(f, mode, Q, val, s);
          if (st != PQ_OK) return st;
          continue;
        }
        const uint32_t pe = f->chunk_page0[(size_t)c * f->nrg + g0 + n];
        for (uint32_t p0 = f->chunk_page0[(size_t)c * f->nrg + g0]; p0 < pe;) {
          uint32_t p1 = p0 + 1;
          auto bytes = [&](uint32_t b) {
            return (f->scratch_prefix[b] - f->scratch_prefix[p0]) + (f->xscratch_prefix[b] - f->xscratch_prefix[p0]);
          };
          while (p1 < pe && bytes(p1 + 1) <= INDEX_WS_CAP / 2) ++p1;
          Plan R;
          st = make_plan(f, 1ull << c, g0, g0 + n, R, true, p0, p1);
          if (st == PQ_OK) st = prefix_plan(f, mode, R, val, s);
          if (st != PQ_OK) return st;
          p0 = p1;
        }
      }
    }
    g0 += n;
  }
  return PQ_OK;
}

static pq_status build_tile_prefix(pq_file f, hipStream_t s) {
  const uint64_t nt = f->total_tiles;
  std::vector<bool> need((size_t)f->ncols, false), need_dlba((size_t)f->ncols, false);
  bool any_dlba = false;
  for (int c = 0; c < f->ncols; ++c) {
    need[(size_t)c] = f->cols[c].type == T_BYTE_ARRAY;
    for (uint32_t p = f->chunk_page0[(size_t)c * f->nrg]; p < f->chunk_page0[(size_t)(c + 1) * f->nrg]; ++p) {
      if (f->pages[p].kind == PAGE_DICT) continue;
      if (f->pages[p].encoding == E_DELTA) need[(size_t)c] = true;
      if (f->pages[p].encoding == E_DLBA && f->cols[c].type == T_BYTE_ARRAY) need_dlba[(size_t)c] = any_dlba = true;
    }
  }
  // the DELTA sums of DELTA_LENGTH_BYTE_ARRAY length streams first: the
  // string-byte pass needs their carries
  if (any_dlba) {
    std::vector<uint64_t> val2(nt, 0);
    pq_status st = prefix_pass(f, 1, need_dlba, val2, s);
    if (st != PQ_OK) return st;
    std::vector<uint64_t> p2(nt + 1, 0);
    for (uint64_t t = 0; t < nt; ++t) p2[t + 1] = p2[t] + val2[t];
    HIP_OR(hipMalloc(&f->d_tpfx2, 8ull * (nt + 1)));
    HIP_OR(hipMemcpy(f->d_tpfx2, p2.data(), 8ull * (nt + 1), hipMemcpyHostToDevice));
    f->fd.tpfx2 = f->d_tpfx2;
    f->device_bytes += 8ull * (nt + 1);
  }
  std::vector<uint64_t> val(nt, 0);
  pq_status st = prefix_pass(f, 0, need, val, s);
  if (st != PQ_OK) return st;
  f->tpfx.assign(nt + 1, 0);
  for (uint64_t t = 0; t < nt; ++t) f->tpfx[t + 1] = f->tpfx[t] + val[t];
  HIP_OR(hipMalloc(&f->d_tpfx, 8ull * (nt + 1)));
  HIP_OR(hipMemcpy(f->d_tpfx, f->tpfx.data(), 8ull * (nt + 1), hipMemcpyHostToDevice));
  f->fd.tpfx = f->d_tpfx;
  return PQ_OK;
}

extern "C" pq_status pq_plan(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end, pq_scan_sizes* out) {
  if (!f || !out) return fail(PQ_EINVAL, "NULL argument");
  Plan P;
  pq_status st = make_plan(f, col_mask, rg_begin, rg_end, P);
  if (st != PQ_OK) return st;
  if (P.cols.size() > MAX_SEGS) return fail(PQ_EUNSUPPORTED, "too many columns");
  out->rows = P.rows;
  out->workspace_bytes = P.ws_total;
  for (int k = 0; k < 64; ++k) out->chars_bytes[k] = 0;
  for (int32_t k : P.str_cols) {
    const ColScan& cs = P.cols[k];
    out->chars_bytes[k] = (int64_t)(f->tpfx[cs.tile_end] - f->tpfx[cs.tile_begin]);
  }
  return PQ_OK;
}

// Checks the caller's output descriptors against a plan and stores their
// pointers in its column table.
static pq_status bind_outputs(Plan& P, const pq_column_out* outs, int32_t n_outs) {
  if ((int32_t)P.cols.size() != n_outs) return fail(PQ_EINVAL, "n_outs (%d) differs from the mask's columns (%d)", n_outs, (int)P.cols.size());
  if (n_outs && !outs) return fail(PQ_EINVAL, "outs is NULL");
  for (size_t k = 0; k < P.cols.size(); ++k) {
    ColScan& cs = P.cols[k];
    const pq_column_out& o = outs[k];
    if (o.validity && ((uintptr_t)o.validity & 3)) return fail(PQ_EINVAL, "column %d: validity must be 4-byte aligned", cs.col);
    if (cs.optional && !o.validity && P.rows > 0) return fail(PQ_EINVAL, "column %d: OPTIONAL column needs a validity buffer", cs.col);
    if (cs.type == T_BYTE_ARRAY) {
      if (!o.offsets) return fail(PQ_EINVAL, "column %d: offsets is NULL", cs.col);
      if (o.chars_capacity && !o.chars) return fail(PQ_EINVAL, "column %d: chars is NULL", cs.col);
      cs.offsets = o.offsets;
      cs.chars = o.chars;
      cs.chars_capacity = o.chars ? o.chars_capacity : 0;
    } else {
      if (P.rows > 0 && !o.values) return fail(PQ_EINVAL, "column %d: values is NULL", cs.col);
      if ((uintptr_t)o.values % (uint64_t)cs.width) return fail(PQ_EINVAL, "column %d: values misaligned", cs.col);
      cs.values = o.values;
    }
    cs.validity = o.validity;
  }
  return PQ_OK;
}

extern "C" pq_status pq_scan(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end, const pq_column_out* outs,
                             int32_t n_outs, void* workspace, uint64_t workspace_bytes, pq_stream stream) {
  if (!f) return fail(PQ_EINVAL, "NULL handle");
  if (f->host) return fail(PQ_EINVAL, "a host-resident file is scanned with pq_scan_streamed");
  Plan P;
  pq_status st = make_plan(f, col_mask, rg_begin, rg_end, P);
  if (st != PQ_OK) return st;
  if (P.cols.size() > MAX_SEGS) return fail(PQ_EUNSUPPORTED, "too many columns");
  if (!workspace) return fail(PQ_EINVAL, "workspace is NULL");
  if (workspace_bytes < P.ws_total) return fail(PQ_ECAPACITY, "workspace smaller than planned (%llu < %llu)",
                                                (unsigned long long)workspace_bytes, (unsigned long long)P.ws_total);
  if (((uintptr_t)workspace & 255) != 0) return fail(PQ_EINVAL, "workspace must be 256-byte aligned");
  st = bind_outputs(P, outs, n_outs);
  if (st != PQ_OK) return st;
  return enqueue(f, P, (uint8_t*)workspace, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// allocation-free scans
// ---------------------------------------------------------------------------
// The workspace of pq_scan_noalloc: a file-scope device array of
// NOALLOC_BYTES on every GPU the library runs on, held until the process
// ends.  Host code never passes its name to a kernel or a copy (that is a
// host-side stand-in); it takes the array's device address, per device,
// from hipGetSymbolAddress on the first call made on that device.
constexpr uint64_t NOALLOC_BYTES = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static uint8_t* g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of the current device's scratch array (nullptr on error,
// with the message set).
static uint8_t* scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    fail(PQ_EHIP, "pq_scan_noalloc: no current device (or device id %d out of range)", dev);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fail(PQ_EHIP, "pq_scan_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
  }
  return g_scratch_ptr[dev];
}

extern "C" pq_status pq_scan_noalloc(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end,
                                     const pq_column_out* outs, int32_t n_outs, pq_stream stream) {
  if (!f) return fail(PQ_EINVAL, "NULL handle");
  if (f->host) return fail(PQ_EINVAL, "a host-resident file is scanned with pq_scan_streamed");
  Plan P;
  pq_status st = make_plan(f, col_mask, rg_begin, rg_end, P);
  if (st != PQ_OK) return st;
  if (P.cols.size() > MAX_SEGS) return fail(PQ_EUNSUPPORTED, "too many columns");
  if (P.ws_total > NOALLOC_BYTES)
    return fail(PQ_ECAPACITY, "pq_scan_noalloc: the scan needs %llu bytes of workspace, above the %llu-byte scratch array "
                "(use pq_scan with a caller workspace)", (unsigned long long)P.ws_total, (unsigned long long)NOALLOC_BYTES);
  st = bind_outputs(P, outs, n_outs);
  if (st != PQ_OK) return st;
  uint8_t* ws = scratch_of_current_device();
  if (!ws) return PQ_EHIP;
  return enqueue(f, P, ws, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// streamed scans of host-resident files
// ---------------------------------------------------------------------------
extern "C" pq_status pq_scan_streamed(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end,
                                      const pq_column_out* outs, int32_t n_outs, void* workspace, uint64_t workspace_bytes,
                                      pq_stream copy_stream, pq_stream stream) {
  if (!f) return fail(PQ_EINVAL, "NULL handle");
  if (!f->host) return fail(PQ_EINVAL, "pq_scan_streamed needs a host-resident file (pq_open_host)");
  Plan P;
  pq_status st = make_plan(f, col_mask, rg_begin, rg_end, P);
  if (st != PQ_OK) return st;
  if (P.cols.size() > MAX_SEGS) return fail(PQ_EUNSUPPORTED, "too many columns");
  if (!workspace) return fail(PQ_EINVAL, "workspace is NULL");
  if (workspace_bytes < P.ws_total) return fail(PQ_ECAPACITY, "workspace smaller than planned (%llu < %llu)",
                                                (unsigned long long)workspace_bytes, (unsigned long long)P.ws_total);
  if (((uintptr_t)workspace & 255) != 0) return fail(PQ_EINVAL, "workspace must be 256-byte aligned");
  st = bind_outputs(P, outs, n_outs);
  if (st != PQ_OK) return st;
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  hipStream_t s = (hipStream_t)stream, cs = (hipStream_t)copy_stream;
  uint32_t* err = reinterpret_cast<uint32_t*>(ws);
  st = upload_header(P, ws, s);
  if (st != PQ_OK) return st;
  const int nrg = rg_end - rg_begin;
  if (nrg == 0 || P.cols.empty()) return enqueue_finish(f, P, reinterpret_cast<ColScan*>(ws + P.ws_cols), ws, err, s);
  // one column table per row group: the file base of its slot
  std::vector<ColScan> tables(P.cols.size() * (size_t)nrg);
  for (int i = 0; i < nrg; ++i)
    for (size_t k = 0; k < P.cols.size(); ++k) {
      ColScan t = P.cols[k];
      t.fd.file = ws + P.ws_stage + (uint64_t)(i % 2) * P.stage_bytes - P.rg_lo[(size_t)i];
      tables[(size_t)i * P.cols.size() + k] = t;
    }
  HIP_OR(hipMemcpyAsync(ws + P.ws_rgcols, tables.data(), sizeof(ColScan) * tables.size(), hipMemcpyHostToDevice, s));
  for (hipEvent_t& e : f->stage_ev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      return fail(PQ_EHIP, "event creation failed");
    }
  hipEvent_t* copied = f->stage_ev;
  hipEvent_t* freed = f->stage_ev + 2;
  // the first slot's copy waits for the upload that precedes it on `stream`
  (void)hipEventRecord(freed[1], s);
  (void)hipStreamWaitEvent(cs, freed[1], 0);
  for (int i = 0; i < nrg && st == PQ_OK; ++i) {
    const int g = rg_begin + i, slot = i % 2;
    if (i >= 2 && hipStreamWaitEvent(cs, freed[slot], 0) != hipSuccess) { st = fail(PQ_EHIP, "stream wait failed"); break; }
    uint8_t* base = ws + P.ws_stage + (uint64_t)slot * P.stage_bytes;
    for (const ColScan& c : P.cols) {
      const ChunkDev& ch = f->chunks[(size_t)c.col * f->nrg + g];
      if (ch.end > ch.start &&
          hipMemcpyAsync(base + (ch.start - P.rg_lo[(size_t)i]), f->host + ch.start, ch.end - ch.start,
                         hipMemcpyHostToDevice, cs) != hipSuccess) {
        st = fail(PQ_EHIP, "row group %d: host-to-device copy failed", g);
        break;
      }
    }
    if (st != PQ_OK) break;
    if (hipEventRecord(copied[slot], cs) != hipSuccess || hipStreamWaitEvent(s, copied[slot], 0) != hipSuccess) {
      st = fail(PQ_EHIP, "event record failed");
      break;
    }
    Plan Pg;  // the launch lists of row group g alone (same column order)
    st = make_plan(f, col_mask, g, g + 1, Pg);
    const ColScan* d_cols = reinterpret_cast<const ColScan*>(ws + P.ws_rgcols + sizeof(ColScan) * P.cols.size() * (size_t)i);
    // (Pg's workspace offsets are not this workspace's: the buckets are P's)
    if (st == PQ_OK) st = enqueue_decompress(f, Pg, d_cols, ws, err, s, P.ws_sord, P.sblk_lanes);
    if (st == PQ_OK) st = enqueue_decode(f, Pg, d_cols, ws, err, s);
    if (st == PQ_OK && hipEventRecord(freed[slot], s) != hipSuccess) st = fail(PQ_EHIP, "event record failed");
  }
  if (st == PQ_OK) st = enqueue_finish(f, P, reinterpret_cast<ColScan*>(ws + P.ws_cols), ws, err, s);
  return st;
}

extern "C" pq_status pq_scan_check(pq_file f, const void* workspace, pq_stream stream) {
  (void)f;
  if (!workspace) {
    // the scratch array of pq_scan_noalloc on the current device
    uint8_t* p = scratch_of_current_device();
    if (!p) return PQ_EHIP;
    return read_err_word(reinterpret_cast<uint32_t*>(p), (hipStream_t)stream);
  }
  return read_err_word(reinterpret_cast<uint32_t*>(const_cast<void*>(workspace)), (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// batched scans
// ---------------------------------------------------------------------------
// The measurement recorder of batched scans (pq_profile(NULL, ...)).
static pq_file_s g_batch_prof;

namespace {

constexpr int NWCLASS = 2, NPCLASS = 3;
static_assert((int)TK_KINDS * NWCLASS * NPCLASS == PQ_TUNE_CLASSES, "work classes");
constexpr uint32_t DEFAULT_TPU = 2, DEFAULT_WPC = 8;
constexpr uint32_t NUM_CUS = 256;  // MI355X compute units (8 XCDs x 32)
// relative cost of one tile per decoder kind (roughly the bytes it moves),
// used only to balance the queues
constexpr uint64_t KIND_COST[TK_KINDS] = {8, 7, 16, 11, 9, 40, 40, 8, 16};

// The decoder kind of a data page's tiles.
uint32_t tile_kind(pq_file f, const PageDev& pg, const ColScan& cs) {
  const bool dict = pg.encoding == E_PLAIN_DICT || pg.encoding == E_RLE_DICT;
  if (cs.type == T_BYTE_ARRAY) return dict && (f->dicts[pg.chunk].flags & DICT_SLOTS) ? TK_STRSLOT : TK_STR;
  if (pg.encoding == E_DELTA) return TK_DELTA;
  if (pg.encoding == E_BSS) return cs.width == 8 ? TK_BSS8 : TK_BSS4;
  if (pg.encoding != E_PLAIN && !dict) return TK_FIXED1;  // its decoder reports the encoding as unsupported
  return (dict ? 1u : 0u) | (cs.width == 8 ? 2u : 0u);
}

uint32_t tune_class(uint32_t kind, const PageDev& pg, uint32_t ntiles) {
  const bool dict_kind = kind == TK_FIXED1 || kind == TK_FIXED3 || kind == TK_STR || kind == TK_STRSLOT;
  const uint32_t w = dict_kind && pg.enc_w > 12 ? 1 : 0;
  const uint32_t pc = ntiles <= 1 ? 0 : (ntiles <= 16 ? 1 : 2);
  return (kind * NWCLASS + w) * NPCLASS + pc;
}

struct BatchPlan {
  std::vector<ColScan> cols;
  std::vector<int32_t> str_cols;
  std::vector<int64_t> chars;  // per column, in request order
  std::vector<Segment> snappy_segs, sblk_segs, edge_segs, prep_segs, dba_segs;
  uint32_t snappy_waves = 0, sblk_lanes = 0, edge_threads = 0, prep_threads = 0, dba_waves = 0;
  // same-kind tile runs: consecutive pages of one column with one decoder
  // and work class
  struct Run { uint32_t cs, t0, t1, kind, cls, chunk; };
  std::vector<Run> runs;
  std::vector<uint32_t> run_file;  // request index of each run (chunk keys are per file)
  std::vector<Run> page_runs;      // one per data page (the per-page form's launches)
  struct SnapPage { uint32_t cs, page, b0, b1; };
  std::vector<SnapPage> snap_pages;  // compressed data pages and their Snappy blocks
  std::vector<std::pair<uint32_t, uint32_t>> dba_pages;  // (column, page) of DELTA_BYTE_ARRAY pages
  uint64_t total_tiles = 0;
  uint64_t ws_cols = 0, ws_which = 0, ws_snappy = 0, ws_sblk = 0, ws_edge = 0, ws_prep = 0, ws_units = 0,
           ws_qbeg = 0, ws_qhead = 0, ws_hdr_end = 0, ws_total = 0, ws_dba = 0;
};

pq_status make_batch_plan(const pq_request* reqs, int32_t n, BatchPlan& P) {
  if (n < 0 || (n > 0 && !reqs)) return fail(PQ_EINVAL, "bad request list");
  uint64_t ncols = 0;
  for (int32_t r = 0; r < n; ++r) {
    if (!reqs[r].file) return fail(PQ_EINVAL, "request %d: NULL file", r);
    if (reqs[r].file->host) return fail(PQ_EINVAL, "request %d: a host-resident file", r);
    ncols += (uint64_t)__builtin_popcountll(reqs[r].col_mask);
  }
  if (ncols >= (1ull << 31)) return fail(PQ_EUNSUPPORTED, "too many columns in one batch");
  // tiles of the whole batch bound the units the header must hold
  uint64_t tiles = 0, snappy_segs = 0;
  for (int32_t r = 0; r < n; ++r) {
    pq_file f = reqs[r].file;
    const pq_request& q = reqs[r];
    if (q.rg_begin < 0 || q.rg_end > f->nrg || q.rg_begin > q.rg_end)
      return fail(PQ_EINVAL, "request %d: bad row-group range [%d, %d)", r, q.rg_begin, q.rg_end);
    if (f->ncols < 64 && (q.col_mask >> f->ncols)) return fail(PQ_EINVAL, "request %d: mask selects missing columns", r);
    for (int c = 0; c < f->ncols; ++c) {
      if (!((q.col_mask >> c) & 1)) continue;
      tiles += f->chunk_tile0[(size_t)c * f->nrg + q.rg_end] - f->chunk_tile0[(size_t)c * f->nrg + q.rg_begin];
      snappy_segs += 1;
    }
  }
  P.total_tiles = tiles;
  uint64_t off = WS_HEADER;
  P.ws_cols = off;
  off = align_up(off + sizeof(ColScan) * (ncols ? ncols : 1), 256);
  P.ws_which = off;
  off = align_up(off + sizeof(int32_t) * (ncols ? ncols : 1), 256);
  P.ws_snappy = off;
  off = align_up(off + sizeof(Segment) * (snappy_segs ? snappy_segs : 1), 256);
  P.ws_sblk = off;
  off = align_up(off + sizeof(Segment) * (snappy_segs ? snappy_segs : 1), 256);
  P.ws_dba = off;
  off = align_up(off + sizeof(Segment) * (snappy_segs ? snappy_segs : 1), 256);
  P.ws_edge = off;
  off = align_up(off + sizeof(Segment) * (ncols ? ncols : 1), 256);
  P.ws_prep = off;
  off = align_up(off + sizeof(Segment) * (ncols ? ncols : 1), 256);
  P.ws_units = off;
  off = align_up(off + sizeof(BUnit) * (tiles ? tiles : 1), 256);
  P.ws_qbeg = off;
  off = align_up(off + sizeof(uint32_t) * (NQUEUE + 1), 256);
  P.ws_qhead = off;
  off = align_up(off + sizeof(uint32_t) * NQUEUE, 256);
  P.ws_hdr_end = off;
  for (int32_t r = 0; r < n; ++r) {
    pq_file f = reqs[r].file;
    const pq_request& q = reqs[r];
    const int64_t rows = f->rg_row0[q.rg_end] - f->rg_row0[q.rg_begin];
    for (int c = 0; c < f->ncols; ++c) {
      if (!((q.col_mask >> c) & 1)) continue;
      ColSetup k;
      col_setup(f, c, q.rg_begin, q.rg_end, rows, off, false, k);
      const ColScan& cs = k.cs;
      const uint32_t idx = (uint32_t)P.cols.size();
      P.chars.push_back(cs.type == T_BYTE_ARRAY ? (int64_t)(f->tpfx[cs.tile_end] - f->tpfx[cs.tile_begin]) : 0);
      if (cs.type == T_BYTE_ARRAY) P.str_cols.push_back((int32_t)idx);
      if (k.sbytes) {
        P.snappy_segs.push_back(Segment{idx, cs.page_begin, cs.page_end, P.snappy_waves});
        P.snappy_waves += cs.page_end - cs.page_begin;
        if (k.b1 > k.b0) {
          P.sblk_segs.push_back(Segment{idx, k.b0, k.b1, P.sblk_lanes});
          P.sblk_lanes += k.b1 - k.b0;
        }
      }
      if (k.xbytes) {
        P.dba_segs.push_back(Segment{idx, cs.page_begin, cs.page_end, P.dba_waves});
        P.dba_waves += cs.page_end - cs.page_begin;
      }
      if (k.nt) {
        if (cs.optional) {
          P.edge_segs.push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.edge_threads});
          P.edge_threads += k.nt;
        } else {
          P.prep_segs.push_back(Segment{idx, cs.tile_begin, cs.tile_end, P.prep_threads});
          P.prep_threads += k.nt;
        }
      }
      for (uint32_t p = cs.page_begin; p < cs.page_end; ++p) {
        const PageDev& pg = f->pages[p];
        if (pg.kind == PAGE_DICT) continue;
        if (pg.scratch_len) {
          const uint32_t nb = (uint32_t)(((uint64_t)pg.scratch_len + SNAP_BLOCK - 1) / SNAP_BLOCK);
          P.snap_pages.push_back(BatchPlan::SnapPage{idx, p, pg.sblk_begin, pg.sblk_begin + nb});
        }
        if (pg.encoding == E_DBA && cs.type == T_BYTE_ARRAY) P.dba_pages.push_back({idx, p});
        const uint32_t nt = (uint32_t)(((uint64_t)(pg.num_values > 0 ? pg.num_values : 0) + TILE_ROWS - 1) / TILE_ROWS);
        if (!nt) continue;
        const uint32_t kind = tile_kind(f, pg, cs), cls = tune_class(kind, pg, nt);
        P.page_runs.push_back(BatchPlan::Run{idx, pg.tile_begin, pg.tile_begin + nt, kind, cls, pg.chunk});
        if (!P.runs.empty()) {
          BatchPlan::Run& b = P.runs.back();
          if (b.cs == idx && b.kind == kind && b.cls == cls && b.t1 == pg.tile_begin && b.chunk == pg.chunk) {
            b.t1 += nt;
            continue;
          }
        }
        P.runs.push_back(BatchPlan::Run{idx, pg.tile_begin, pg.tile_begin + nt, kind, cls, pg.chunk});
        P.run_file.push_back((uint32_t)r);
      }
      P.cols.push_back(cs);
    }
  }
  P.ws_total = std::max<uint64_t>(off, 256);
  return PQ_OK;
}

// Work units and queue bounds of a plan under a schedule.  With one queue
// per XCD, the chunks (all units of one column chunk) are dealt to the
// queues longest first, each to the least loaded one, so that a chunk's
// dictionary is gathered through one XCD's L2; a queue then serves its
// costliest units first.
void make_units(const BatchPlan& P, const pq_tuning& T, std::vector<BUnit>& units, uint32_t qbeg[NQUEUE + 1]) {
  struct U { BUnit u; uint64_t cost; uint64_t key; };
  std::vector<U> all;
  all.reserve(P.total_tiles);
  for (size_t i = 0; i < P.runs.size(); ++i) {
    const BatchPlan::Run& r = P.runs[i];
    uint32_t tpu = T.tiles_per_unit[r.cls] ? T.tiles_per_unit[r.cls] : DEFAULT_TPU;
    tpu = std::min<uint32_t>(std::max<uint32_t>(tpu, 1), 64);
    for (uint32_t t = r.t0; t < r.t1; t += tpu) {
      const uint32_t t1 = std::min(r.t1, t + tpu);
      all.push_back(U{BUnit{r.cs, t, t1, r.kind}, (uint64_t)(t1 - t) * KIND_COST[r.kind],
                      ((uint64_t)P.run_file[i] << 32) | r.chunk});
    }
  }
  units.clear();
  const int nq = T.queues == 1 ? 1 : NQUEUE;
  if (nq == 1) {
    for (const U& u : all) units.push_back(u.u);
    qbeg[0] = 0;
    for (int q = 1; q <= NQUEUE; ++q) qbeg[q] = (uint32_t)units.size();
    return;
  }
  // chunks, longest first, to the least loaded queue
  std::vector<std::pair<uint64_t, uint64_t>> chunks;  // (key, cost)
  {
    std::vector<U> sorted = all;
    std::stable_sort(sorted.begin(), sorted.end(), [](const U& a, const U& b) { return a.key < b.key; });
    for (size_t i = 0; i < sorted.size();) {
      size_t j = i;
      uint64_t c = 0;
      while (j < sorted.size() && sorted[j].key == sorted[i].key) c += sorted[j++].cost;
      chunks.push_back({sorted[i].key, c});
      i = j;
    }
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const std::pair<uint64_t, uint64_t>& a, const std::pair<uint64_t, uint64_t>& b) {
    return a.second > b.second;
  });
  std::vector<uint64_t> load(NQUEUE, 0);
  std::vector<std::pair<uint64_t, int>> qof;  // chunk key -> queue
  qof.reserve(chunks.size());
  for (const auto& ch : chunks) {
    int best = 0;
    for (int q = 1; q < NQUEUE; ++q)
      if (load[q] < load[best]) best = q;
    load[best] += ch.second;
    qof.push_back({ch.first, best});
  }
  std::sort(qof.begin(), qof.end());
  std::vector<std::vector<U>> per(NQUEUE);
  for (const U& u : all) {
    auto it = std::lower_bound(qof.begin(), qof.end(), std::make_pair(u.key, -1));
    per[it->second].push_back(u);
  }
  qbeg[0] = 0;
  for (int q = 0; q < NQUEUE; ++q) {
    std::stable_sort(per[q].begin(), per[q].end(), [](const U& a, const U& b) { return a.cost > b.cost; });
    for (const U& u : per[q]) units.push_back(u.u);
    qbeg[q + 1] = (uint32_t)units.size();
  }
}

SegTable seg_table(const std::vector<Segment>& v, uint8_t* ws, uint64_t ws_off) {
  SegTable t;
  memset(&t, 0, sizeof(t));
  t.n = (int32_t)v.size();
  if (v.size() <= (size_t)MAX_SEGS) {
    for (size_t i = 0; i < v.size(); ++i) t.s[i] = v[i];
  } else {
    t.ptr = reinterpret_cast<const Segment*>(ws + ws_off);
  }
  return t;
}

pq_status bind_batch_outputs(const pq_request* reqs, int32_t n, BatchPlan& P) {
  size_t k = 0;
  for (int32_t r = 0; r < n; ++r) {
    const int nc = __builtin_popcountll(reqs[r].col_mask);
    if (nc && !reqs[r].outs) return fail(PQ_EINVAL, "request %d: outs is NULL", r);
    Plan one;
    one.rows = P.cols[k].rows;
    one.cols.assign(P.cols.begin() + (long)k, P.cols.begin() + (long)k + nc);
    if (nc) {
      pq_status st = bind_outputs(one, reqs[r].outs, nc);
      if (st != PQ_OK) return st;
      std::copy(one.cols.begin(), one.cols.end(), P.cols.begin() + (long)k);
    }
    k += (size_t)nc;
  }
  return PQ_OK;
}

pq_status enqueue_batch(const BatchPlan& P, const pq_tuning& T, uint8_t* ws, hipStream_t s) {
  pq_file prof = &g_batch_prof;
  uint32_t* err = reinterpret_cast<uint32_t*>(ws);
  std::vector<BUnit> units;
  uint32_t qbeg[NQUEUE + 1];
  const bool per_page = T.form == PQ_FORM_PER_PAGE;
  if (!per_page) make_units(P, T, units, qbeg);
  // the header: error word, column table, string columns, segment tables,
  // units, queue bounds and heads, in one copy
  std::vector<uint8_t> hdr(P.ws_hdr_end, 0);
  auto put = [&](uint64_t at, const void* src, size_t n) { if (n) memcpy(hdr.data() + at, src, n); };
  put(P.ws_cols, P.cols.data(), sizeof(ColScan) * P.cols.size());
  put(P.ws_which, P.str_cols.data(), sizeof(int32_t) * P.str_cols.size());
  put(P.ws_snappy, P.snappy_segs.data(), sizeof(Segment) * P.snappy_segs.size());
  put(P.ws_sblk, P.sblk_segs.data(), sizeof(Segment) * P.sblk_segs.size());
  put(P.ws_dba, P.dba_segs.data(), sizeof(Segment) * P.dba_segs.size());
  put(P.ws_edge, P.edge_segs.data(), sizeof(Segment) * P.edge_segs.size());
  put(P.ws_prep, P.prep_segs.data(), sizeof(Segment) * P.prep_segs.size());
  if (!per_page) {
    put(P.ws_units, units.data(), sizeof(BUnit) * units.size());
    put(P.ws_qbeg, qbeg, sizeof(qbeg));
  }
  HIP_OR(hipMemcpyAsync(ws, hdr.data(), hdr.size(), hipMemcpyHostToDevice, s));
  const ColScan* d_cols = reinterpret_cast<const ColScan*>(ws + P.ws_cols);
  // decompression
  if (!per_page) {
    if (P.snappy_waves) {
      ProfScope ps_(prof, KP_SNAPPY, s);
      hipLaunchKernelGGL(k_snappy, dim3(P.snappy_waves), dim3(64), 0, s, d_cols, seg_table(P.snappy_segs, ws, P.ws_snappy),
                         ws, 0, err);
      HIP_OR(hipGetLastError());
    }
    if (P.sblk_lanes) {
      ProfScope ps_(prof, KP_SNAPPY_BLK, s);
      hipLaunchKernelGGL(k_snappy_blk, dim3((P.sblk_lanes + 4 * SNAP_LANES - 1) / (4 * SNAP_LANES)), dim3(256), 0, s,
                         d_cols, seg_table(P.sblk_segs, ws, P.ws_sblk), (const uint32_t*)nullptr, 0u, ws, err, 0);
      HIP_OR(hipGetLastError());
    }
  } else {
    // one launch per compressed page: the page-sequential decoder (which
    // leaves at once for a page with a block index) and the block decoder
    for (const BatchPlan::SnapPage& sp : P.snap_pages) {
      {
        ProfScope ps_(prof, KP_SNAPPY, s);
        std::vector<Segment> one{Segment{sp.cs, sp.page, sp.page + 1, 0}};
        hipLaunchKernelGGL(k_snappy, dim3(1), dim3(64), 0, s, d_cols, make_segs(one), ws, 0, err);
        HIP_OR(hipGetLastError());
      }
      if (sp.b1 > sp.b0) {
        ProfScope ps_(prof, KP_SNAPPY_BLK, s);
        std::vector<Segment> one{Segment{sp.cs, sp.b0, sp.b1, 0}};
        hipLaunchKernelGGL(k_snappy_blk, dim3((sp.b1 - sp.b0 + 4 * SNAP_LANES - 1) / (4 * SNAP_LANES)), dim3(256), 0, s,
                           d_cols, make_segs(one), (const uint32_t*)nullptr, 0u, ws, err, 0);
        HIP_OR(hipGetLastError());
      }
    }
  }
  // DELTA_BYTE_ARRAY pages to the PLAIN layout (after their decompression)
  if (!per_page) {
    if (P.dba_waves) {
      hipLaunchKernelGGL(k_dba, dim3(P.dba_waves), dim3(64), 0, s, d_cols, seg_table(P.dba_segs, ws, P.ws_dba), ws,
                         (const uint8_t*)nullptr, (uint8_t*)nullptr, (PageDev*)nullptr, 1, err);
      HIP_OR(hipGetLastError());
    }
  } else {
    for (const auto& dp : P.dba_pages) {
      std::vector<Segment> one{Segment{dp.first, dp.second, dp.second + 1, 0}};
      hipLaunchKernelGGL(k_dba, dim3(1), dim3(64), 0, s, d_cols, make_segs(one), ws, (const uint8_t*)nullptr,
                         (uint8_t*)nullptr, (PageDev*)nullptr, 1, err);
      HIP_OR(hipGetLastError());
    }
  }
  if (!P.str_cols.empty()) {
    ProfScope ps_(prof, KP_STR_TOTAL, s);
    hipLaunchKernelGGL(k_str_total, dim3(((uint32_t)P.str_cols.size() + 63) / 64), dim3(64), 0, s, d_cols,
                       reinterpret_cast<const int32_t*>(ws + P.ws_which), (int32_t)P.str_cols.size(), err);
    HIP_OR(hipGetLastError());
  }
  if (!per_page) {
    if (!units.empty()) {
      ProfScope ps_(prof, KP_BATCH, s);
      const uint32_t wpc = T.waves_per_cu > 0 ? (uint32_t)std::min(T.waves_per_cu, 16) : DEFAULT_WPC;
      const uint32_t wgs = std::max<uint32_t>(1, std::min<uint32_t>(NUM_CUS * wpc / 4, ((uint32_t)units.size() + 3) / 4));
      hipLaunchKernelGGL(k_batch, dim3(wgs), dim3(256), 0, s, ws, d_cols,
                         reinterpret_cast<const BUnit*>(ws + P.ws_units), reinterpret_cast<const uint32_t*>(ws + P.ws_qbeg),
                         reinterpret_cast<uint32_t*>(ws + P.ws_qhead), err);
      HIP_OR(hipGetLastError());
    }
  } else {
    if (P.prep_threads) {
      for (const Segment& sg : P.prep_segs) {
        ProfScope ps_(prof, KP_PREP, s);
        std::vector<Segment> one{Segment{sg.cs, sg.t0, sg.t1, 0}};
        hipLaunchKernelGGL(k_prep, dim3((sg.t1 - sg.t0 + 255) / 256), dim3(256), 0, s, d_cols, make_segs(one));
        HIP_OR(hipGetLastError());
      }
    }
    for (const BatchPlan::Run& r : P.page_runs) {
      std::vector<Segment> one{Segment{r.cs, r.t0, r.t1, 0}};
      const uint32_t wg = (r.t1 - r.t0 + 3) / 4;
      switch (r.kind) {
        case TK_FIXED0: case TK_FIXED1: case TK_FIXED2: case TK_FIXED3: case TK_BSS4: case TK_BSS8: {
          const int K = r.kind == TK_BSS4 ? FX_BSS : r.kind == TK_BSS8 ? (FX_BSS | FX_WIDE) : (int)r.kind;
          ProfScope ps_(prof, KP_FIXED0 + K, s);
          hipLaunchKernelGGL(fixed_kernel(K), dim3(wg), dim3(256), 0, s, ws, d_cols, make_segs(one), err);
          break;
        }
        case TK_DELTA: {
          ProfScope ps_(prof, KP_DELTA, s);
          hipLaunchKernelGGL(k_decode_delta, dim3(wg), dim3(256), 0, s, ws, d_cols, make_segs(one), err);
          break;
        }
        default: {
          ProfScope ps_(prof, r.kind == TK_STRSLOT ? KP_STR_SLOTS : KP_STR, s);
          hipLaunchKernelGGL(r.kind == TK_STRSLOT ? k_decode_str<true> : k_decode_str<false>, dim3(wg), dim3(256), 0, s,
                             ws, d_cols, make_segs(one), err);
        }
      }
      HIP_OR(hipGetLastError());
    }
  }
  if (P.edge_threads) {
    ProfScope ps_(prof, KP_EDGES, s);
    hipLaunchKernelGGL(k_edges, dim3((P.edge_threads + 255) / 256), dim3(256), 0, s, ws, d_cols,
                       seg_table(P.edge_segs, ws, P.ws_edge));
    HIP_OR(hipGetLastError());
  }
  return PQ_OK;
}

}  // namespace

extern "C" pq_status pq_tuning_default(pq_tuning* out) {
  if (!out) return fail(PQ_EINVAL, "NULL argument");
  memset(out, 0, sizeof(*out));
  out->form = PQ_FORM_BATCHED;
  out->waves_per_cu = (int32_t)DEFAULT_WPC;
  out->queues = NQUEUE;
  for (int c = 0; c < PQ_TUNE_CLASSES; ++c) out->tiles_per_unit[c] = (uint8_t)DEFAULT_TPU;
  return PQ_OK;
}

extern "C" pq_status pq_plan_batch(const pq_request* reqs, int32_t n, uint64_t* workspace_bytes, int64_t* chars_bytes,
                                   int32_t n_chars) {
  if (!workspace_bytes) return fail(PQ_EINVAL, "NULL argument");
  BatchPlan P;
  pq_status st = make_batch_plan(reqs, n, P);
  if (st != PQ_OK) return st;
  *workspace_bytes = P.ws_total;
  if (chars_bytes) {
    if ((size_t)n_chars < P.chars.size()) return fail(PQ_EINVAL, "chars_bytes holds %d entries, the batch has %zu columns", n_chars, P.chars.size());
    for (size_t k = 0; k < P.chars.size(); ++k) chars_bytes[k] = P.chars[k];
  }
  return PQ_OK;
}

static pq_status scan_batch(const pq_request* reqs, int32_t n, const pq_tuning* tuning, void* workspace,
                            uint64_t workspace_bytes, hipStream_t s, BatchPlan* cached) {
  BatchPlan local;
  BatchPlan& P = cached ? *cached : local;
  if (!cached) {
    pq_status st = make_batch_plan(reqs, n, P);
    if (st != PQ_OK) return st;
    st = bind_batch_outputs(reqs, n, P);
    if (st != PQ_OK) return st;
  }
  if (!workspace) return fail(PQ_EINVAL, "workspace is NULL");
  if (workspace_bytes < P.ws_total) return fail(PQ_ECAPACITY, "workspace smaller than planned (%llu < %llu)",
                                                (unsigned long long)workspace_bytes, (unsigned long long)P.ws_total);
  if (((uintptr_t)workspace & 255) != 0) return fail(PQ_EINVAL, "workspace must be 256-byte aligned");
  pq_tuning T;
  pq_tuning_default(&T);
  if (tuning) T = *tuning;
  if (T.form != PQ_FORM_BATCHED && T.form != PQ_FORM_PER_PAGE) return fail(PQ_EINVAL, "unknown form %d", T.form);
  return enqueue_batch(P, T, (uint8_t*)workspace, s);
}

extern "C" pq_status pq_scan_batch(const pq_request* reqs, int32_t n, const pq_tuning* tuning, void* workspace,
                                   uint64_t workspace_bytes, pq_stream stream) {
  return scan_batch(reqs, n, tuning, workspace, workspace_bytes, (hipStream_t)stream, nullptr);
}

extern "C" pq_status pq_autotune_batch(const pq_request* reqs, int32_t n, void* workspace, uint64_t workspace_bytes,
                                       pq_stream stream, int32_t reps, pq_tuning* best, double* best_ms,
                                       double* default_ms) {
  if (!best) return fail(PQ_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  BatchPlan P;
  pq_status st = make_batch_plan(reqs, n, P);
  if (st != PQ_OK) return st;
  st = bind_batch_outputs(reqs, n, P);
  if (st != PQ_OK) return st;
  if (reps < 1) reps = 3;
  hipEvent_t e0, e1;
  HIP_OR(hipEventCreate(&e0));
  HIP_OR(hipEventCreate(&e1));
  auto timed = [&](const pq_tuning& T, double& ms) -> pq_status {
    std::vector<double> v;
    for (int r = 0; r < reps; ++r) {
      HIP_OR(hipEventRecord(e0, s));
      pq_status st2 = scan_batch(reqs, n, &T, workspace, workspace_bytes, s, &P);
      if (st2 != PQ_OK) return st2;
      HIP_OR(hipEventRecord(e1, s));
      HIP_OR(hipEventSynchronize(e1));
      float f = 0;
      HIP_OR(hipEventElapsedTime(&f, e0, e1));
      v.push_back(f);
    }
    std::sort(v.begin(), v.end());
    ms = v[v.size() / 2];
    return read_err_word(reinterpret_cast<uint32_t*>(workspace), s);
  };
  pq_tuning cur;
  pq_tuning_default(&cur);
  double cur_ms = 0;
  pq_status rs = timed(cur, cur_ms);  // warms the caches and the code too
  if (rs == PQ_OK) rs = timed(cur, cur_ms);
  if (rs != PQ_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return rs; }
  if (default_ms) *default_ms = cur_ms;
  auto consider = [&](const pq_tuning& T) -> pq_status {
    double ms = 0;
    pq_status st2 = timed(T, ms);
    if (st2 != PQ_OK) return st2;
    if (ms < cur_ms) { cur = T; cur_ms = ms; }
    return PQ_OK;
  };
  // 1. queue layout, 2. waves per CU
  for (int q : {1}) {
    pq_tuning T = cur;
    T.queues = q;
    if (rs == PQ_OK) rs = consider(T);
  }
  for (int w : {4, 12, 16}) {
    pq_tuning T = cur;
    T.waves_per_cu = w;
    if (rs == PQ_OK) rs = consider(T);
  }
  // 3. tiles per unit of each class present, the classes with most tiles first
  std::vector<std::pair<uint64_t, int>> cls(PQ_TUNE_CLASSES);
  for (int c = 0; c < PQ_TUNE_CLASSES; ++c) cls[c] = {0, c};
  for (const BatchPlan::Run& r : P.runs) cls[r.cls].first += r.t1 - r.t0;
  std::stable_sort(cls.begin(), cls.end(), [](const std::pair<uint64_t, int>& a, const std::pair<uint64_t, int>& b) { return a.first > b.first; });
  for (const auto& c : cls) {
    if (!c.first) break;
    for (int tpu : {1, 4, 8, 16}) {
      pq_tuning T = cur;
      T.tiles_per_unit[c.second] = (uint8_t)tpu;
      if (rs == PQ_OK) rs = consider(T);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rs != PQ_OK) return rs;
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return PQ_OK;
}

extern "C" pq_status pq_column_bytes(pq_file f, int32_t col, uint64_t* data_bytes, uint64_t* dict_bytes) {
  if (!f || col < 0 || col >= f->ncols) return fail(PQ_EINVAL, "bad column");
  uint64_t d = 0, k = 0;
  const uint32_t q0 = (uint32_t)(col * f->nrg), q1 = (uint32_t)((col + 1) * f->nrg);
  for (uint32_t p = f->chunk_page0[q0]; p < f->chunk_page0[q1]; ++p) {
    if (f->pages[p].kind == PAGE_DICT) k += f->pages[p].comp_size;
    else d += f->pages[p].comp_size;
  }
  if (data_bytes) *data_bytes = d;
  if (dict_bytes) *dict_bytes = k;
  return PQ_OK;
}

extern "C" pq_status pq_column_encodings(pq_file f, int32_t col, uint32_t* mask) {
  if (!f || !mask || col < 0 || col >= f->ncols) return fail(PQ_EINVAL, "bad argument");
  uint32_t m = 0;
  const uint32_t q0 = (uint32_t)(col * f->nrg), q1 = (uint32_t)((col + 1) * f->nrg);
  for (uint32_t p = f->chunk_page0[q0]; p < f->chunk_page0[q1]; ++p)
    if (f->pages[p].kind != PAGE_DICT && f->pages[p].encoding < 32) m |= 1u << f->pages[p].encoding;
  *mask = m;
  return PQ_OK;
}

static pq_file prof_of(pq_file f) { return f ? f : &g_batch_prof; }

extern "C" pq_status pq_copy_probe(void* dst, const void* src, uint64_t bytes, pq_stream stream) {
  if (!bytes) return PQ_OK;
  if (!dst || !src) return fail(PQ_EINVAL, "NULL buffer");
  const uint64_t chunks = bytes >> 4;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(16384, (chunks + 1023) / 1024));
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream, static_cast<uint8_t*>(dst),
                     static_cast<const uint8_t*>(src), bytes);
  HIP_OR(hipGetLastError());
  return PQ_OK;
}

extern "C" pq_status pq_profile(pq_file f, int32_t enable) {
  f = prof_of(f);
  for (auto& r : f->recs) { f->event_pool.push_back(r.a); f->event_pool.push_back(r.b); }
  f->recs.clear();
  for (int k = 0; k < NKERN; ++k) { f->prof_ms[k] = 0; f->prof_n[k] = 0; }
  f->profiling = enable != 0;
  return PQ_OK;
}

extern "C" pq_status pq_profile_read(pq_file f, pq_kernel_time* out, int32_t capacity, int32_t* n) {
  f = prof_of(f);
  if (!n) return fail(PQ_EINVAL, "NULL argument");
  for (auto& r : f->recs) {
    HIP_OR(hipEventSynchronize(r.b));
    float ms = 0;
    HIP_OR(hipEventElapsedTime(&ms, r.a, r.b));
    f->prof_ms[r.kernel] += ms;
    f->prof_n[r.kernel] += 1;
    f->event_pool.push_back(r.a);
    f->event_pool.push_back(r.b);
  }
  f->recs.clear();
  int32_t k = 0;
  for (int j = 0; j < NKERN; ++j) {
    if (!f->prof_n[j]) continue;
    if (out && k < capacity) {
      memset(out[k].name, 0, sizeof(out[k].name));
      strncpy(out[k].name, kKernelNames[j], sizeof(out[k].name) - 1);
      out[k].launches = f->prof_n[j];
      out[k].total_ms = f->prof_ms[j];
    }
    ++k;
  }
  *n = k;
  return PQ_OK;
}
