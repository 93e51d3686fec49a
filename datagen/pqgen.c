/*
 * pqgen.c -- seeded synthetic Parquet writer.
 *
 * Test and benchmark INPUT GENERATOR.  It produces Parquet files whose knobs
 * are the four the paper varies (row-group size, page size, encoding,
 * compression; Sec. 1 and Sec. 3), filled with counter-based pseudo-random
 * values, and it can regenerate the decoded columns directly from the seeds
 * (the plain definition of what any correct reader must return).
 *
 * It shares no code with the CPU oracle (oracle/) or with the GPU reader
 * (paper_2602_17335_amd/csrc/): both only ever see the bytes written here.
 * Nothing in this file decodes Parquet; it only encodes.
 *
 * Format facts follow the public Apache Parquet format description (file
 * layout, Thrift compact footer, page headers, the RLE/bit-packed hybrid,
 * DELTA_BINARY_PACKED, PLAIN) and the public Snappy raw-format description.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* public structs (mirrored by ctypes in datagen/__init__.py)           */
/* ------------------------------------------------------------------ */

enum { PT_INT32 = 1, PT_INT64 = 2, PT_DOUBLE = 5, PT_BYTE_ARRAY = 6 };
enum { EN_PLAIN = 0, EN_PLAIN_DICT = 2, EN_RLE = 3, EN_DELTA = 5, EN_DLBA = 6, EN_DBA = 7, EN_RLE_DICT = 8, EN_BSS = 9 };
enum {
  D_UNIFORM = 0,  /* ints: U[lo, hi); double: U[dlo, dhi)                  */
  D_ZIPF = 1,     /* rank in [1, hi] with exponent zipf_s                    */
  D_SORTED = 2,   /* lo + U[0, hi) start, then + U{1..gap_max} per row        */
  D_DICTVALS = 3, /* hi distinct random values, picked uniformly per row     */
  D_STRINGS = 4,  /* hi distinct strings (0: a new string per row)           */
  D_CONST = 5,    /* every row = lo                                          */
  D_RUNS = 6      /* runs: value changes every run_len rows (U[lo,hi))       */
};

typedef struct {
  int32_t ptype;
  int32_t encoding; /* data-page encoding: PLAIN, RLE_DICTIONARY, PLAIN_DICTIONARY, DELTA */
  int32_t optional;
  int32_t dist;
  double null_prob;
  int64_t lo, hi;
  double dlo, dhi;
  double zipf_s;
  int32_t str_min, str_max;
  int32_t gap_max;
  int32_t run_len;
} pqg_col;

typedef struct {
  uint64_t seed;
  int64_t num_rows;
  int64_t rg_rows;
  int64_t page_bytes;     /* target encoded (pre-compression) bytes per data page */
  int64_t dict_cap;       /* 0: unlimited; else PLAIN fallback when dict would exceed */
  int32_t codec;          /* 0 UNCOMPRESSED, 1 SNAPPY */
  int32_t page_version;   /* 1 or 2 */
  int32_t delta_block;    /* values per DELTA block (multiple of 128) */
  int32_t delta_mini;     /* miniblocks per block */
  int32_t max_bp_groups;  /* cap on groups of 8 in one bit-packed run (<= 63) */
  int32_t rle_min;        /* repeat count at which the hybrid encoder switches to RLE */
  int32_t ncols;
  int32_t nthreads;
  int32_t snappy_skip;    /* 0: greedy matcher; 1: literal-only Snappy streams;
                             2: greedy matcher, every tag form in turn */
  int32_t index_width;    /* dictionary index bit width when wider than the minimum (0: minimal) */
  int32_t encoding_search; /* 1: per chunk, the candidate encoding of smallest encoded size */
  int32_t min_saving_pct;  /* >0: a chunk stays uncompressed unless Snappy saves more than this many percent */
} pqg_spec;

/* ------------------------------------------------------------------ */
/* counter-based random numbers (splitmix64 finaliser)                  */
/* ------------------------------------------------------------------ */

static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static inline uint64_t draw(uint64_t stream, uint64_t i) { return mix64(stream ^ mix64(i)); }
static inline uint64_t below(uint64_t r, uint64_t n) { return (uint64_t)(((unsigned __int128)r * n) >> 64); }

typedef struct {
  uint64_t s_null, s_val, s_len, s_chr, s_start, s_dict;
} streams_t;

static streams_t col_streams(uint64_t seed, int col) {
  uint64_t cs = seed ^ ((uint64_t)(col + 1) * 0x9E3779B97F4A7C15ull);
  streams_t s;
  s.s_null = mix64(cs ^ 0x11);
  s.s_val = mix64(cs ^ 0x22);
  s.s_len = mix64(cs ^ 0x33);
  s.s_chr = mix64(cs ^ 0x44);
  s.s_start = mix64(cs ^ 0x55);
  s.s_dict = mix64(cs ^ 0x66);
  return s;
}

/* Zipf CDF table, one per column that needs it (built lazily, shared). */
typedef struct {
  int64_t n;
  double s;
  double* cdf;
} zipf_t;

static zipf_t* zipf_build(int64_t n, double s) {
  zipf_t* z = (zipf_t*)malloc(sizeof(zipf_t));
  z->n = n;
  z->s = s;
  z->cdf = (double*)malloc(sizeof(double) * (size_t)n);
  double acc = 0;
  for (int64_t k = 1; k <= n; ++k) {
    acc += pow((double)k, -s);
    z->cdf[k - 1] = acc;
  }
  for (int64_t k = 0; k < n; ++k) z->cdf[k] /= acc;
  z->cdf[n - 1] = 1.0;
  return z;
}
static int64_t zipf_rank(const zipf_t* z, uint64_t r) {
  double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);
  int64_t lo = 0, hi = z->n - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (z->cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo + 1;
}

/* Generated row: validity + either a 64-bit payload or a string id. */
typedef struct {
  const pqg_col* c;
  streams_t st;
  zipf_t* zipf;
  uint64_t start;
} colgen_t;

static void colgen_init(colgen_t* g, const pqg_spec* sp, const pqg_col* c, int col) {
  g->c = c;
  g->st = col_streams(sp->seed, col);
  g->zipf = NULL;
  if (c->dist == D_ZIPF) g->zipf = zipf_build(c->hi, c->zipf_s);
  g->start = 0;
  if (c->dist == D_SORTED) g->start = (uint64_t)c->lo + below(draw(g->st.s_start, 0), (uint64_t)(c->hi > 0 ? c->hi : 1));
}
static void colgen_free(colgen_t* g) {
  if (g->zipf) { free(g->zipf->cdf); free(g->zipf); }
}

static inline int row_valid(const colgen_t* g, int64_t row) {
  if (!g->c->optional || g->c->null_prob <= 0) return 1;
  if (g->c->null_prob >= 1.0) return 0;
  double t = g->c->null_prob * 18446744073709551616.0;
  return (double)draw(g->st.s_null, (uint64_t)row) >= t;
}

static inline uint64_t double_bits(double d) { uint64_t u; memcpy(&u, &d, 8); return u; }

/* value of distinct entry d for D_DICTVALS */
static inline uint64_t dict_entry(const colgen_t* g, uint64_t d) {
  const pqg_col* c = g->c;
  uint64_t r = draw(g->st.s_dict, d);
  if (c->ptype == PT_DOUBLE) return double_bits(c->dlo + (double)(r >> 11) * (1.0 / 9007199254740992.0) * (c->dhi - c->dlo));
  if (c->ptype == PT_INT32) return (uint64_t)(uint32_t)r;
  return r;
}

/* Generator id of a row (for dictionary-style dists) or the raw value.
   For D_SORTED this needs the running key, so it is handled by callers. */
static inline uint64_t row_id(const colgen_t* g, int64_t row) {
  const pqg_col* c = g->c;
  uint64_t r = draw(g->st.s_val, (uint64_t)row);
  switch (c->dist) {
    case D_ZIPF: return (uint64_t)(zipf_rank(g->zipf, r) - 1);
    case D_DICTVALS: return below(r, (uint64_t)c->hi);
    case D_STRINGS: return c->hi > 0 ? below(r, (uint64_t)c->hi) : (uint64_t)row;
    case D_RUNS: return (uint64_t)(row / (c->run_len > 0 ? c->run_len : 1));
    default: return r;
  }
}

/* 64-bit payload for a fixed-width row given its id (not D_SORTED). */
static inline uint64_t row_value_from_id(const colgen_t* g, uint64_t id) {
  const pqg_col* c = g->c;
  switch (c->dist) {
    case D_UNIFORM:
      if (c->ptype == PT_DOUBLE) return double_bits(c->dlo + (double)(id >> 11) * (1.0 / 9007199254740992.0) * (c->dhi - c->dlo));
      return (uint64_t)(c->lo + (int64_t)below(id, (uint64_t)(c->hi - c->lo)));
    case D_ZIPF: return id + 1;
    case D_DICTVALS: return dict_entry(g, id);
    case D_CONST: return (uint64_t)c->lo;
    case D_RUNS: {
      uint64_t r = draw(g->st.s_dict, id);
      if (c->ptype == PT_DOUBLE) return double_bits(c->dlo + (double)(r >> 11) * (1.0 / 9007199254740992.0) * (c->dhi - c->dlo));
      return (uint64_t)(c->lo + (int64_t)below(r, (uint64_t)(c->hi - c->lo)));
    }
    default: return id;
  }
}

static inline int string_len(const colgen_t* g, uint64_t d) {
  const pqg_col* c = g->c;
  int span = c->str_max - c->str_min + 1;
  if (span < 1) span = 1;
  return c->str_min + (int)below(draw(g->st.s_len, d), (uint64_t)span);
}
static inline void string_fill(const colgen_t* g, uint64_t d, uint8_t* dst, int len) {
  uint64_t w = 0;
  for (int k = 0; k < len; ++k) {
    if ((k & 7) == 0) w = draw(g->st.s_chr, d * 64 + (uint64_t)(k >> 3));
    dst[k] = (uint8_t)('a' + (uint8_t)(w & 0xff) % 26);
    w >>= 8;
  }
}

/* gap for D_SORTED */
static inline uint64_t sorted_gap(const colgen_t* g, int64_t row) {
  int gm = g->c->gap_max > 0 ? g->c->gap_max : 1;
  return 1 + below(draw(g->st.s_val, (uint64_t)row), (uint64_t)gm);
}

/* ------------------------------------------------------------------ */
/* byte buffer                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
  uint8_t* p;
  size_t n, cap;
} buf_t;

static void buf_reserve(buf_t* b, size_t extra) {
  if (b->n + extra <= b->cap) return;
  size_t nc = b->cap ? b->cap : 256;
  while (nc < b->n + extra) nc *= 2;
  b->p = (uint8_t*)realloc(b->p, nc);
  b->cap = nc;
}
static inline void put_u8(buf_t* b, uint8_t v) { buf_reserve(b, 1); b->p[b->n++] = v; }
static inline void put_bytes(buf_t* b, const void* s, size_t n) { buf_reserve(b, n); memcpy(b->p + b->n, s, n); b->n += n; }
static inline void put_u32le(buf_t* b, uint32_t v) { uint8_t t[4] = {(uint8_t)v, (uint8_t)(v >> 8), (uint8_t)(v >> 16), (uint8_t)(v >> 24)}; put_bytes(b, t, 4); }
static inline void put_uleb(buf_t* b, uint64_t v) {
  do { uint8_t c = v & 0x7f; v >>= 7; if (v) c |= 0x80; put_u8(b, c); } while (v);
}
static inline uint64_t zz64(int64_t v) { return ((uint64_t)v << 1) ^ (uint64_t)(v >> 63); }
static void buf_free(buf_t* b) { free(b->p); b->p = NULL; b->n = b->cap = 0; }

/* ------------------------------------------------------------------ */
/* Thrift compact-protocol writer                                       */
/* ------------------------------------------------------------------ */

enum { TT_TRUE = 1, TT_FALSE = 2, TT_I32 = 5, TT_I64 = 6, TT_BIN = 8, TT_LIST = 9, TT_STRUCT = 12 };

typedef struct {
  buf_t* b;
  int16_t last[32];
  int depth;
} tw_t;

static void tw_init(tw_t* t, buf_t* b) { t->b = b; t->depth = 0; t->last[0] = 0; }
static void tw_field(tw_t* t, int id, int type) {
  int d = id - t->last[t->depth];
  if (d > 0 && d <= 15) put_u8(t->b, (uint8_t)((d << 4) | type));
  else { put_u8(t->b, (uint8_t)type); put_uleb(t->b, zz64(id)); }
  t->last[t->depth] = (int16_t)id;
}
static void tw_i32(tw_t* t, int id, int32_t v) { tw_field(t, id, TT_I32); put_uleb(t->b, zz64(v)); }
static void tw_i64(tw_t* t, int id, int64_t v) { tw_field(t, id, TT_I64); put_uleb(t->b, zz64(v)); }
static void tw_bin(tw_t* t, int id, const char* s, size_t n) { tw_field(t, id, TT_BIN); put_uleb(t->b, n); put_bytes(t->b, s, n); }
static void tw_bool(tw_t* t, int id, int v) { tw_field(t, id, v ? TT_TRUE : TT_FALSE); }
static void tw_struct_begin(tw_t* t, int id) { tw_field(t, id, TT_STRUCT); t->last[++t->depth] = 0; }
static void tw_struct_end(tw_t* t) { put_u8(t->b, 0); t->depth--; }
static void tw_list_begin(tw_t* t, int id, int etype, size_t n) {
  tw_field(t, id, TT_LIST);
  if (n < 15) put_u8(t->b, (uint8_t)((n << 4) | etype));
  else { put_u8(t->b, (uint8_t)(0xF0 | etype)); put_uleb(t->b, n); }
}
static void tw_elem_begin(tw_t* t) { t->last[++t->depth] = 0; }
static void tw_elem_end(tw_t* t) { put_u8(t->b, 0); t->depth--; }

/* ------------------------------------------------------------------ */
/* encoders                                                             */
/* ------------------------------------------------------------------ */

/* bit-pack `n` values of width w (LSB-first), padding the last group of 8 */
static void bitpack(buf_t* b, const uint64_t* v, size_t n, int w) {
  size_t ngroups = (n + 7) / 8;
  size_t nbytes = ngroups * (size_t)w;
  buf_reserve(b, nbytes + 16);
  uint8_t* o = b->p + b->n;
  memset(o, 0, nbytes);
  unsigned __int128 acc = 0;
  int bits = 0;
  size_t pos = 0;
  uint64_t mask = w >= 64 ? ~0ull : ((1ull << w) - 1);
  for (size_t i = 0; i < ngroups * 8; ++i) {
    uint64_t x = i < n ? (v[i] & mask) : 0;
    acc |= (unsigned __int128)x << bits;
    bits += w;
    while (bits >= 8) { o[pos++] = (uint8_t)acc; acc >>= 8; bits -= 8; }
  }
  if (bits > 0) o[pos++] = (uint8_t)acc;
  b->n += nbytes;
}

typedef struct {
  int max_groups;
  int rle_min;
} hyb_opts;

/* RLE / bit-packed hybrid encoder: bit-packed runs of whole groups of 8,
   switching to an RLE run when a value repeats at least rle_min times and
   the pending literal values form whole groups. RLE runs may have any
   length (not a multiple of 8). */
static void hybrid_encode(buf_t* b, const uint64_t* v, size_t n, int w, hyb_opts o) {
  size_t i = 0;
  size_t lit0 = 0, nlit = 0; /* pending literal values are v[lit0 .. lit0+nlit) */
  int vbytes = (w + 7) / 8;
  size_t maxlit = (size_t)o.max_groups * 8;
  while (i < n) {
    size_t r = 1;
    while (i + r < n && v[i + r] == v[i]) ++r;
    if (r >= (size_t)o.rle_min && (nlit % 8) == 0) {
      /* flush literal values */
      while (nlit > 0) {
        size_t take = nlit < maxlit ? nlit : maxlit;
        put_uleb(b, ((uint64_t)(take / 8) << 1) | 1);
        bitpack(b, v + lit0, take, w);
        lit0 += take; nlit -= take;
      }
      put_uleb(b, (uint64_t)r << 1);
      for (int k = 0; k < vbytes; ++k) put_u8(b, (uint8_t)(v[i] >> (8 * k)));
      i += r;
      lit0 = i;
      continue;
    }
    size_t take = 1;
    if (r >= (size_t)o.rle_min) take = 8 - (nlit % 8); /* complete the group first */
    if (nlit == 0) lit0 = i;
    nlit += take;
    i += take;
    if (nlit == maxlit) {
      put_uleb(b, ((uint64_t)(nlit / 8) << 1) | 1);
      bitpack(b, v + lit0, nlit, w);
      lit0 = i; nlit = 0;
    }
  }
  while (nlit > 0) {
    size_t take = nlit < maxlit ? nlit : maxlit;
    size_t groups = (take + 7) / 8;
    put_uleb(b, ((uint64_t)groups << 1) | 1);
    bitpack(b, v + lit0, take, w);
    lit0 += take; nlit -= take;
  }
}

static int bits_needed(uint64_t x) { int w = 0; while (x) { ++w; x >>= 1; } return w; }

/* DELTA_BINARY_PACKED over n values (wrapping at 32 bits when is32). */
static void delta_encode(buf_t* b, const uint64_t* v, size_t n, int is32, int block, int mini) {
  put_uleb(b, (uint64_t)block);
  put_uleb(b, (uint64_t)mini);
  put_uleb(b, (uint64_t)n);
  int64_t first = is32 ? (int64_t)(int32_t)(uint32_t)(n ? v[0] : 0) : (int64_t)(n ? v[0] : 0);
  put_uleb(b, zz64(first));
  if (n <= 1) return;
  size_t nd = n - 1;
  int per_mini = block / mini;
  uint64_t* d = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)block);
  uint64_t* u = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)block);
  for (size_t b0 = 0; b0 < nd; b0 += (size_t)block) {
    size_t cnt = nd - b0 < (size_t)block ? nd - b0 : (size_t)block;
    int64_t mn = INT64_MAX;
    for (size_t k = 0; k < cnt; ++k) {
      uint64_t cur = v[b0 + k + 1], prev = v[b0 + k];
      int64_t dd;
      if (is32) dd = (int64_t)(int32_t)((uint32_t)cur - (uint32_t)prev);
      else dd = (int64_t)(cur - prev);
      d[k] = (uint64_t)dd;
      if (dd < mn) mn = dd;
    }
    put_uleb(b, zz64(mn));
    int widths[256];
    int nm_used = (int)((cnt + (size_t)per_mini - 1) / (size_t)per_mini);
    for (int m = 0; m < mini; ++m) {
      widths[m] = 0;
      if (m >= nm_used) continue;
      uint64_t mx = 0;
      for (int k = 0; k < per_mini; ++k) {
        size_t idx = (size_t)m * (size_t)per_mini + (size_t)k;
        if (idx >= cnt) break;
        uint64_t x = is32 ? (uint64_t)(uint32_t)((uint32_t)d[idx] - (uint32_t)mn) : d[idx] - (uint64_t)mn;
        if (x > mx) mx = x;
      }
      widths[m] = bits_needed(mx);
    }
    for (int m = 0; m < mini; ++m) put_u8(b, (uint8_t)widths[m]);
    for (int m = 0; m < nm_used; ++m) {
      for (int k = 0; k < per_mini; ++k) {
        size_t idx = (size_t)m * (size_t)per_mini + (size_t)k;
        if (idx < cnt) u[k] = is32 ? (uint64_t)(uint32_t)((uint32_t)d[idx] - (uint32_t)mn) : d[idx] - (uint64_t)mn;
        else u[k] = 0;
      }
      bitpack(b, u, (size_t)per_mini, widths[m]);
    }
  }
  free(d);
  free(u);
}

/* ------------------------------------------------------------------ */
/* Snappy raw-format compressor (greedy hash matcher, 64 KiB fragments) */
/* ------------------------------------------------------------------ */

static void sn_literal(buf_t* b, const uint8_t* s, size_t n) {
  while (n > 0) {
    size_t take = n > 0xFFFFFFFFull ? 0xFFFFFFFFull : n;
    size_t l = take - 1;
    if (l < 60) put_u8(b, (uint8_t)(l << 2));
    else if (l < 256) { put_u8(b, 60 << 2); put_u8(b, (uint8_t)l); }
    else if (l < 65536) { put_u8(b, 61 << 2); put_u8(b, (uint8_t)l); put_u8(b, (uint8_t)(l >> 8)); }
    else if (l < (1u << 24)) { put_u8(b, 62 << 2); put_u8(b, (uint8_t)l); put_u8(b, (uint8_t)(l >> 8)); put_u8(b, (uint8_t)(l >> 16)); }
    else { put_u8(b, 63 << 2); put_u32le(b, (uint32_t)l); }
    put_bytes(b, s, take);
    s += take; n -= take;
  }
}
static void sn_copy1(buf_t* b, size_t off, size_t len) {
  if (off < 2048 && len >= 4 && len <= 11) {
    put_u8(b, (uint8_t)(((off >> 8) << 5) | ((len - 4) << 2) | 1));
    put_u8(b, (uint8_t)off);
  } else {
    put_u8(b, (uint8_t)(((len - 1) << 2) | 2));
    put_u8(b, (uint8_t)off); put_u8(b, (uint8_t)(off >> 8));
  }
}
static void sn_copy(buf_t* b, size_t off, size_t len) {
  while (len >= 68) { sn_copy1(b, off, 64); len -= 64; }
  if (len > 64) { sn_copy1(b, off, 60); len -= 60; }
  sn_copy1(b, off, len);
}
/* mode 2: the same elements written in every legal form in turn (a fixture
   for decoders): literal lengths in the tag or in 1-4 length bytes (more than
   needed), copies with a 1-, 2- or 4-byte offset */
static void sn_literal_v(buf_t* b, const uint8_t* s, size_t n, unsigned* ctr) {
  while (n > 0) {
    size_t take = n > 0xFFFFFFFFull ? 0xFFFFFFFFull : n;
    size_t l = take - 1;
    unsigned nb = l < 60 ? 0 : l < 256 ? 1 : l < 65536 ? 2 : l < (1u << 24) ? 3 : 4;
    unsigned k = (*ctr)++ % 5;
    if (k > nb) nb = k;
    if (nb == 0) {
      put_u8(b, (uint8_t)(l << 2));
    } else {
      put_u8(b, (uint8_t)((59 + nb) << 2));
      for (unsigned i = 0; i < nb; ++i) put_u8(b, (uint8_t)(l >> (8 * i)));
    }
    put_bytes(b, s, take);
    s += take; n -= take;
  }
}
static void sn_copy_v(buf_t* b, size_t off, size_t len, unsigned* ctr) {
  while (len > 0) {
    size_t take = len > 64 ? 64 : len;
    unsigned k = (*ctr)++ % 3;
    if (k == 0 && off < 2048 && take >= 4 && take <= 11) {
      put_u8(b, (uint8_t)(((off >> 8) << 5) | ((take - 4) << 2) | 1));
      put_u8(b, (uint8_t)off);
    } else if (k <= 1 && off < 65536) {
      put_u8(b, (uint8_t)(((take - 1) << 2) | 2));
      put_u8(b, (uint8_t)off); put_u8(b, (uint8_t)(off >> 8));
    } else {
      put_u8(b, (uint8_t)(((take - 1) << 2) | 3));
      put_u32le(b, (uint32_t)off);
    }
    len -= take;
  }
}

static inline uint32_t ld32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }

/* mode 0: greedy matcher; 1: one literal; 2: greedy matcher, the elements in
   every tag form in turn */
void pqg_snappy_compress(const uint8_t* src, size_t n, buf_t* b, int mode) {
  put_uleb(b, n);
  if (mode == 1) { if (n) sn_literal(b, src, n); return; }
  unsigned ctr_l = 0, ctr_c = 0;
  int32_t* table = (int32_t*)malloc(sizeof(int32_t) * (1 << 14));
  for (size_t f0 = 0; f0 < n; f0 += 65536) {
    size_t f1 = f0 + 65536 < n ? f0 + 65536 : n;
    memset(table, 0, sizeof(int32_t) * (1 << 14));
    size_t ip = f0, lit = f0;
    while (ip + 4 <= f1) {
      uint32_t x = ld32(src + ip);
      uint32_t h = (x * 0x1e35a7bdu) >> 18;
      int32_t cand = table[h] - 1;
      table[h] = (int32_t)(ip - f0) + 1;
      if (cand >= 0 && (size_t)cand + f0 < ip && ld32(src + f0 + cand) == x) {
        size_t c = f0 + (size_t)cand;
        size_t len = 4;
        while (ip + len < f1 && src[c + len] == src[ip + len]) ++len;
        if (mode == 2) {
          if (ip > lit) sn_literal_v(b, src + lit, ip - lit, &ctr_l);
          sn_copy_v(b, ip - c, len, &ctr_c);
        } else {
          if (ip > lit) sn_literal(b, src + lit, ip - lit);
          sn_copy(b, ip - c, len);
        }
        ip += len;
        lit = ip;
      } else {
        ++ip;
      }
    }
    if (f1 > lit) {
      if (mode == 2) sn_literal_v(b, src + lit, f1 - lit, &ctr_l);
      else sn_literal(b, src + lit, f1 - lit);
    }
  }
  free(table);
}

/* exported wrapper for tests: returns malloc'd buffer */
uint8_t* pqg_snappy(const uint8_t* src, size_t n, int mode, size_t* out_len) {
  buf_t b = {0};
  pqg_snappy_compress(src, n, &b, mode);
  *out_len = b.n;
  return b.p;
}

/* ------------------------------------------------------------------ */
/* dictionary builder                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
  /* id-keyed map: generator id -> dictionary index (first occurrence order) */
  int32_t* by_id;
  int64_t id_space;
  /* value-keyed open addressing map (for dists without small id space) */
  uint64_t* keys;
  int32_t* vals;
  size_t hcap;
  /* dictionary content */
  uint64_t* entries; /* 64-bit payload or string id */
  int64_t n, cap;
  int64_t plain_bytes;
} dict_t;

static void dict_init(dict_t* d, int64_t id_space) {
  memset(d, 0, sizeof(*d));
  if (id_space > 0) {
    d->id_space = id_space;
    d->by_id = (int32_t*)malloc(sizeof(int32_t) * (size_t)id_space);
    memset(d->by_id, 0xff, sizeof(int32_t) * (size_t)id_space);
  } else {
    d->hcap = 1024;
    d->keys = (uint64_t*)malloc(sizeof(uint64_t) * d->hcap);
    d->vals = (int32_t*)malloc(sizeof(int32_t) * d->hcap);
    memset(d->vals, 0xff, sizeof(int32_t) * d->hcap);
  }
}
static void dict_free(dict_t* d) { free(d->by_id); free(d->keys); free(d->vals); free(d->entries); }
static void dict_push(dict_t* d, uint64_t e) {
  if (d->n == d->cap) { d->cap = d->cap ? d->cap * 2 : 1024; d->entries = (uint64_t*)realloc(d->entries, sizeof(uint64_t) * (size_t)d->cap); }
  d->entries[d->n++] = e;
}
static void dict_rehash(dict_t* d) {
  size_t nc = d->hcap * 2;
  uint64_t* nk = (uint64_t*)malloc(sizeof(uint64_t) * nc);
  int32_t* nv = (int32_t*)malloc(sizeof(int32_t) * nc);
  memset(nv, 0xff, sizeof(int32_t) * nc);
  for (size_t i = 0; i < d->hcap; ++i) {
    if (d->vals[i] < 0) continue;
    size_t h = (size_t)mix64(d->keys[i]) & (nc - 1);
    while (nv[h] >= 0) h = (h + 1) & (nc - 1);
    nk[h] = d->keys[i]; nv[h] = d->vals[i];
  }
  free(d->keys); free(d->vals);
  d->keys = nk; d->vals = nv; d->hcap = nc;
}
/* Look up key; returns index or -1 when absent (does not insert). */
static int64_t dict_find(dict_t* d, uint64_t key) {
  if (d->by_id) return d->by_id[key];
  size_t h = (size_t)mix64(key) & (d->hcap - 1);
  while (d->vals[h] >= 0) { if (d->keys[h] == key) return d->vals[h]; h = (h + 1) & (d->hcap - 1); }
  return -1;
}
static int64_t dict_insert(dict_t* d, uint64_t key, uint64_t entry, int64_t entry_plain_bytes) {
  int64_t idx = d->n;
  if (d->by_id) d->by_id[key] = (int32_t)idx;
  else {
    if ((size_t)(d->n + 1) * 2 > d->hcap) dict_rehash(d);
    size_t h = (size_t)mix64(key) & (d->hcap - 1);
    while (d->vals[h] >= 0) h = (h + 1) & (d->hcap - 1);
    d->keys[h] = key; d->vals[h] = (int32_t)idx;
  }
  dict_push(d, entry);
  d->plain_bytes += entry_plain_bytes;
  return idx;
}

/* ------------------------------------------------------------------ */
/* chunk encoding                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
  buf_t bytes;          /* dictionary page (if any) followed by data pages */
  int64_t dict_page_rel;/* -1 if no dictionary page */
  int64_t data_page_rel;
  int64_t uncompressed_total;
  int64_t num_values;
  int encs[4];
  int nencs;
  int64_t npages;
  int codec;            /* the chunk's codec (a chunk whose compression saves too little is left uncompressed) */
} chunk_out_t;

typedef struct {
  const pqg_spec* sp;
  const pqg_col* cols;
  colgen_t* gens;
  int64_t* sorted_base; /* per rg: running key before the rg's first row (for D_SORTED cols), [col][rg] */
  int nrg;
  chunk_out_t* outs;    /* [rg][col] */
  int64_t next_task;
  pthread_mutex_t mu;
  int err;
} job_t;

static int ptype_width(int t) { return t == PT_INT32 ? 4 : 8; }

static void add_enc(chunk_out_t* co, int e) {
  for (int i = 0; i < co->nencs; ++i) if (co->encs[i] == e) return;
  co->encs[co->nencs++] = e;
}

typedef struct {
  int64_t nrows;
  uint8_t* valid;    /* per row */
  uint64_t* v;       /* per row: 64-bit payload or string id (null rows: 0) */
} rows_t;

static void write_page_header_v1(buf_t* b, int ptype_is_dict, int32_t unc, int32_t comp, int32_t nvals, int enc, int dict_enc) {
  tw_t t; tw_init(&t, b);
  if (ptype_is_dict) {
    tw_i32(&t, 1, 2);
    tw_i32(&t, 2, unc);
    tw_i32(&t, 3, comp);
    tw_struct_begin(&t, 7);
    tw_i32(&t, 1, nvals);
    tw_i32(&t, 2, dict_enc);
    tw_struct_end(&t);
  } else {
    tw_i32(&t, 1, 0);
    tw_i32(&t, 2, unc);
    tw_i32(&t, 3, comp);
    tw_struct_begin(&t, 5);
    tw_i32(&t, 1, nvals);
    tw_i32(&t, 2, enc);
    tw_i32(&t, 3, EN_RLE);
    tw_i32(&t, 4, EN_RLE);
    tw_struct_end(&t);
  }
  put_u8(b, 0);
}

static void write_page_header_v2(buf_t* b, int32_t unc, int32_t comp, int32_t nvals, int32_t nnulls, int enc, int32_t def_len, int is_compressed) {
  tw_t t; tw_init(&t, b);
  tw_i32(&t, 1, 3);
  tw_i32(&t, 2, unc);
  tw_i32(&t, 3, comp);
  tw_struct_begin(&t, 8);
  tw_i32(&t, 1, nvals);
  tw_i32(&t, 2, nnulls);
  tw_i32(&t, 3, nvals);
  tw_i32(&t, 4, enc);
  tw_i32(&t, 5, def_len);
  tw_i32(&t, 6, 0);
  if (!is_compressed) tw_bool(&t, 7, 0);
  tw_struct_end(&t);
  put_u8(b, 0);
}

/* encode values (non-null only) of rows [r0, r1) with `enc` into vb */
static void encode_values(buf_t* vb, const colgen_t* g, const rows_t* R, int64_t r0, int64_t r1, int enc, const dict_t* dict, int idx_w, const pqg_spec* sp) {
  const pqg_col* c = g->c;
  int64_t nnn = 0;
  for (int64_t r = r0; r < r1; ++r) nnn += R->valid[r];
  if (enc == EN_PLAIN) {
    if (c->ptype == PT_BYTE_ARRAY) {
      for (int64_t r = r0; r < r1; ++r) {
        if (!R->valid[r]) continue;
        int len = string_len(g, R->v[r]);
        buf_reserve(vb, (size_t)len + 4);
        put_u32le(vb, (uint32_t)len);
        string_fill(g, R->v[r], vb->p + vb->n, len);
        vb->n += (size_t)len;
      }
    } else {
      int w = ptype_width(c->ptype);
      buf_reserve(vb, (size_t)(nnn * w));
      for (int64_t r = r0; r < r1; ++r) {
        if (!R->valid[r]) continue;
        uint64_t x = R->v[r];
        memcpy(vb->p + vb->n, &x, (size_t)w); /* little-endian host */
        vb->n += (size_t)w;
      }
    }
  } else if (enc == EN_RLE_DICT || enc == EN_PLAIN_DICT) {
    uint64_t* idx = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnn > 0 ? nnn : 1));
    int64_t k = 0;
    for (int64_t r = r0; r < r1; ++r) {
      if (!R->valid[r]) continue;
      idx[k++] = (uint64_t)dict_find((dict_t*)dict, R->v[r]);
    }
    put_u8(vb, (uint8_t)idx_w);
    hyb_opts o = {sp->max_bp_groups, sp->rle_min};
    hybrid_encode(vb, idx, (size_t)nnn, idx_w, o);
    free(idx);
  } else if (enc == EN_DELTA) {
    uint64_t* vals = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnn > 0 ? nnn : 1));
    int64_t k = 0;
    for (int64_t r = r0; r < r1; ++r) if (R->valid[r]) vals[k++] = R->v[r];
    delta_encode(vb, vals, (size_t)nnn, c->ptype == PT_INT32, sp->delta_block, sp->delta_mini);
    free(vals);
  } else if (enc == EN_BSS) {
    /* w streams of nnn bytes: stream b holds byte b of every value */
    int w = ptype_width(c->ptype);
    buf_reserve(vb, (size_t)(nnn * w));
    uint8_t* o = vb->p + vb->n;
    int64_t k = 0;
    for (int64_t r = r0; r < r1; ++r) {
      if (!R->valid[r]) continue;
      uint64_t x = R->v[r];
      for (int b = 0; b < w; ++b) o[(size_t)b * (size_t)nnn + (size_t)k] = (uint8_t)(x >> (8 * b));
      ++k;
    }
    vb->n += (size_t)(nnn * w);
  } else if (enc == EN_DLBA || enc == EN_DBA) {
    /* strings: lengths (DLBA) or prefix lengths against the previous string
       of the page and suffix lengths (DBA) as DELTA_BINARY_PACKED, then the
       (suffix) bytes */
    uint64_t* pre = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnn > 0 ? nnn : 1));
    uint64_t* len = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nnn > 0 ? nnn : 1));
    buf_t chars = {0};
    uint8_t* prev = (uint8_t*)malloc(1u << 16);
    uint8_t* cur = (uint8_t*)malloc(1u << 16);
    int prev_len = 0;
    int64_t k = 0;
    for (int64_t r = r0; r < r1; ++r) {
      if (!R->valid[r]) continue;
      int l = string_len(g, R->v[r]);
      string_fill(g, R->v[r], cur, l);
      int p = 0;
      if (enc == EN_DBA) {
        while (p < l && p < prev_len && cur[p] == prev[p]) ++p;
      }
      pre[k] = (uint64_t)p;
      len[k] = (uint64_t)(l - p);
      put_bytes(&chars, cur + p, (size_t)(l - p));
      memcpy(prev, cur, (size_t)l);
      prev_len = l;
      ++k;
    }
    if (enc == EN_DBA) delta_encode(vb, pre, (size_t)nnn, 1, sp->delta_block, sp->delta_mini);
    delta_encode(vb, len, (size_t)nnn, 1, sp->delta_block, sp->delta_mini);
    put_bytes(vb, chars.p, chars.n);
    buf_free(&chars);
    free(pre);
    free(len);
    free(prev);
    free(cur);
  }
}

static void encode_defs(buf_t* db, const rows_t* R, int64_t r0, int64_t r1, const pqg_spec* sp) {
  int64_t n = r1 - r0;
  uint64_t* d = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) d[i] = R->valid[r0 + i];
  hyb_opts o = {sp->max_bp_groups, sp->rle_min};
  hybrid_encode(db, d, (size_t)n, 1, o);
  free(d);
}

/* emit one data page for rows [r0, r1) */
static void emit_data_page(chunk_out_t* co, const colgen_t* g, const rows_t* R, int64_t r0, int64_t r1, int enc, const dict_t* dict, int idx_w, const pqg_spec* sp) {
  const pqg_col* c = g->c;
  buf_t db = {0}, vb = {0};
  int64_t nnull = 0;
  for (int64_t r = r0; r < r1; ++r) nnull += !R->valid[r];
  if (c->optional) encode_defs(&db, R, r0, r1, sp);
  encode_values(&vb, g, R, r0, r1, enc, dict, idx_w, sp);
  int32_t nvals = (int32_t)(r1 - r0);
  if (sp->page_version == 2) {
    buf_t cv = {0};
    const uint8_t* vp = vb.p; size_t vn = vb.n;
    if (sp->codec == 1) { pqg_snappy_compress(vb.p, vb.n, &cv, sp->snappy_skip); vp = cv.p; vn = cv.n; }
    int32_t unc = (int32_t)(db.n + vb.n), comp = (int32_t)(db.n + vn);
    write_page_header_v2(&co->bytes, unc, comp, nvals, (int32_t)nnull, enc, (int32_t)db.n, sp->codec == 1);
    put_bytes(&co->bytes, db.p, db.n);
    put_bytes(&co->bytes, vp, vn);
    co->uncompressed_total += unc;
    buf_free(&cv);
  } else {
    buf_t body = {0};
    if (c->optional) { put_u32le(&body, (uint32_t)db.n); put_bytes(&body, db.p, db.n); }
    put_bytes(&body, vb.p, vb.n);
    if (sp->codec == 1) {
      buf_t cb = {0};
      pqg_snappy_compress(body.p, body.n, &cb, sp->snappy_skip);
      write_page_header_v1(&co->bytes, 0, (int32_t)body.n, (int32_t)cb.n, nvals, enc, 0);
      put_bytes(&co->bytes, cb.p, cb.n);
      buf_free(&cb);
    } else {
      write_page_header_v1(&co->bytes, 0, (int32_t)body.n, (int32_t)body.n, nvals, enc, 0);
      put_bytes(&co->bytes, body.p, body.n);
    }
    co->uncompressed_total += (int64_t)body.n;
    buf_free(&body);
  }
  co->npages++;
  add_enc(co, enc);
  buf_free(&db); buf_free(&vb);
}

/* rows per page from a sample encode */
static int64_t rows_per_page(const colgen_t* g, const rows_t* R, int64_t r0, int64_t r1, int enc, const dict_t* dict, int idx_w, const pqg_spec* sp) {
  int64_t n = r1 - r0;
  if (n <= 0) return 1;
  int64_t s = n < 16384 ? n : 16384;
  buf_t db = {0}, vb = {0};
  if (g->c->optional) encode_defs(&db, R, r0, r0 + s, sp);
  encode_values(&vb, g, R, r0, r0 + s, enc, dict, idx_w, sp);
  double bpr = (double)(db.n + vb.n + (g->c->optional ? 4 : 0)) / (double)s;
  buf_free(&db); buf_free(&vb);
  if (bpr <= 0) bpr = 0.01;
  double rp = (double)sp->page_bytes / bpr;
  if (rp < 1) rp = 1;
  if (rp > 2e9) rp = 2e9;
  return (int64_t)rp;
}

/* Encoded bytes of a whole chunk's values with encoding `enc` (one page; a
   dictionary encoding counts its dictionary page), or -1 when `enc` does
   not apply to the column. */
static int64_t chunk_encoded_size(const colgen_t* g, const rows_t* R, int64_t nr, int enc, const pqg_spec* sp) {
  const pqg_col* c = g->c;
  buf_t vb = {0};
  int64_t extra = 0;
  if (enc == EN_RLE_DICT) {
    dict_t d;
    int64_t id_space = (c->ptype == PT_BYTE_ARRAY && c->dist == D_STRINGS && c->hi > 0) ? c->hi : 0;
    dict_init(&d, id_space);
    for (int64_t i = 0; i < nr; ++i) {
      if (!R->valid[i] || dict_find(&d, R->v[i]) >= 0) continue;
      int64_t eb = c->ptype == PT_BYTE_ARRAY ? 4 + string_len(g, R->v[i]) : ptype_width(c->ptype);
      dict_insert(&d, R->v[i], R->v[i], eb);
    }
    int w = d.n <= 1 ? 0 : bits_needed((uint64_t)(d.n - 1));
    extra = d.plain_bytes;
    encode_values(&vb, g, R, 0, nr, enc, &d, w, sp);
    dict_free(&d);
  } else {
    encode_values(&vb, g, R, 0, nr, enc, NULL, 0, sp);
  }
  int64_t n = (int64_t)vb.n + extra;
  buf_free(&vb);
  return n;
}

static void encode_chunk_with(job_t* J, int rg, int col, const pqg_spec* sp);

/* One column chunk; with a minimum Snappy saving, a chunk whose compressed
   pages save too little is written again uncompressed. */
static void encode_chunk(job_t* J, int rg, int col) {
  const pqg_spec* sp = J->sp;
  encode_chunk_with(J, rg, col, sp);
  chunk_out_t* co = &J->outs[(size_t)rg * (size_t)sp->ncols + (size_t)col];
  co->codec = sp->codec;
  if (sp->codec == 1 && sp->min_saving_pct > 0) {
    const int64_t comp = (int64_t)co->bytes.n, unc = co->uncompressed_total;
    if ((double)comp > (double)unc * (1.0 - sp->min_saving_pct / 100.0)) {
      pqg_spec plain = *sp;
      plain.codec = 0;
      buf_free(&co->bytes);
      encode_chunk_with(J, rg, col, &plain);
      co->codec = 0;
    }
  }
}

static void encode_chunk_with(job_t* J, int rg, int col, const pqg_spec* sp) {
  const pqg_col* c = &J->cols[col];
  const colgen_t* g = &J->gens[col];
  chunk_out_t* co = &J->outs[(size_t)rg * (size_t)sp->ncols + (size_t)col];
  int64_t row0 = (int64_t)rg * sp->rg_rows;
  int64_t nr = sp->num_rows - row0 < sp->rg_rows ? sp->num_rows - row0 : sp->rg_rows;
  memset(co, 0, sizeof(*co));
  co->dict_page_rel = -1;
  co->num_values = nr;

  /* 1. generate rows */
  rows_t R;
  R.nrows = nr;
  R.valid = (uint8_t*)malloc((size_t)(nr > 0 ? nr : 1));
  R.v = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nr > 0 ? nr : 1));
  uint64_t key_run = c->dist == D_SORTED ? (uint64_t)J->sorted_base[(size_t)col * (size_t)J->nrg + (size_t)rg] : 0;
  for (int64_t i = 0; i < nr; ++i) {
    int64_t row = row0 + i;
    R.valid[i] = (uint8_t)row_valid(g, row);
    uint64_t x;
    if (c->dist == D_SORTED) {
      key_run += sorted_gap(g, row);
      x = key_run;
      if (c->ptype == PT_INT32) x = (uint64_t)(uint32_t)x;
    } else if (c->ptype == PT_BYTE_ARRAY) {
      x = row_id(g, row);
    } else {
      x = row_value_from_id(g, row_id(g, row));
      if (c->ptype == PT_INT32) x = (uint64_t)(uint32_t)x;
    }
    R.v[i] = R.valid[i] ? x : 0;
  }

  /* the chunk's encoding: the column's, or with the encoding search the
     candidate of smallest encoded size (PLAIN first on ties) */
  int cenc = c->encoding;
  if (sp->encoding_search) {
    int cands[4], nc = 0;
    cands[nc++] = EN_PLAIN;
    cands[nc++] = EN_RLE_DICT;
    if (c->ptype == PT_BYTE_ARRAY) { cands[nc++] = EN_DLBA; cands[nc++] = EN_DBA; }
    else {
      if (c->ptype == PT_INT32 || c->ptype == PT_INT64) cands[nc++] = EN_DELTA;
      cands[nc++] = EN_BSS;
    }
    int64_t best = -1;
    for (int i = 0; i < nc; ++i) {
      int64_t z = chunk_encoded_size(g, &R, nr, cands[i], sp);
      if (z >= 0 && (best < 0 || z < best)) { best = z; cenc = cands[i]; }
    }
  }

  /* 2. dictionary (built in first-occurrence order) */
  int is_dict = (cenc == EN_RLE_DICT || cenc == EN_PLAIN_DICT);
  dict_t dict;
  int64_t fallback = nr; /* rows >= fallback are PLAIN */
  int idx_w = 0;
  if (is_dict) {
    int64_t id_space = 0;
    if (c->ptype == PT_BYTE_ARRAY && c->dist == D_STRINGS && c->hi > 0) id_space = c->hi;
    dict_init(&dict, id_space);
    for (int64_t i = 0; i < nr; ++i) {
      if (!R.valid[i]) continue;
      uint64_t key = R.v[i];
      if (dict_find(&dict, key) >= 0) continue;
      int64_t eb = c->ptype == PT_BYTE_ARRAY ? 4 + string_len(g, key) : ptype_width(c->ptype);
      if (sp->dict_cap > 0 && dict.plain_bytes + eb > sp->dict_cap) { fallback = i; break; }
      dict_insert(&dict, key, key, eb);
    }
    idx_w = dict.n <= 1 ? 0 : bits_needed((uint64_t)(dict.n - 1));
    if (sp->index_width > idx_w && sp->index_width <= 32) idx_w = sp->index_width;
  }

  /* 3. dictionary page */
  if (is_dict) {
    buf_t dp = {0};
    for (int64_t k = 0; k < dict.n; ++k) {
      uint64_t e = dict.entries[k];
      if (c->ptype == PT_BYTE_ARRAY) {
        int len = string_len(g, e);
        buf_reserve(&dp, (size_t)len + 4);
        put_u32le(&dp, (uint32_t)len);
        string_fill(g, e, dp.p + dp.n, len);
        dp.n += (size_t)len;
      } else {
        put_bytes(&dp, &e, (size_t)ptype_width(c->ptype));
      }
    }
    co->dict_page_rel = (int64_t)co->bytes.n;
    int dict_enc = cenc == EN_PLAIN_DICT ? EN_PLAIN_DICT : EN_PLAIN;
    if (sp->codec == 1) {
      buf_t cb = {0};
      pqg_snappy_compress(dp.p, dp.n, &cb, sp->snappy_skip);
      write_page_header_v1(&co->bytes, 1, (int32_t)dp.n, (int32_t)cb.n, (int32_t)dict.n, 0, dict_enc);
      put_bytes(&co->bytes, cb.p, cb.n);
      buf_free(&cb);
    } else {
      write_page_header_v1(&co->bytes, 1, (int32_t)dp.n, (int32_t)dp.n, (int32_t)dict.n, 0, dict_enc);
      put_bytes(&co->bytes, dp.p, dp.n);
    }
    co->uncompressed_total += (int64_t)dp.n;
    add_enc(co, dict_enc);
    buf_free(&dp);
  }
  co->data_page_rel = (int64_t)co->bytes.n;

  /* 4. data pages */
  int64_t r = 0;
  if (is_dict && fallback > 0) {
    int64_t rpp = rows_per_page(g, &R, 0, fallback, cenc, &dict, idx_w, sp);
    while (r < fallback) {
      int64_t e = r + rpp < fallback ? r + rpp : fallback;
      emit_data_page(co, g, &R, r, e, cenc, &dict, idx_w, sp);
      r = e;
    }
  }
  int rest_enc = is_dict ? EN_PLAIN : cenc;
  if (r < nr || nr == 0) {
    int64_t rpp = rows_per_page(g, &R, r, nr, rest_enc, NULL, 0, sp);
    if (nr == 0) emit_data_page(co, g, &R, 0, 0, rest_enc, NULL, 0, sp);
    while (r < nr) {
      int64_t e = r + rpp < nr ? r + rpp : nr;
      emit_data_page(co, g, &R, r, e, rest_enc, NULL, 0, sp);
      r = e;
    }
  }
  add_enc(co, EN_RLE);
  if (is_dict) dict_free(&dict);
  free(R.valid);
  free(R.v);
}

static void* worker(void* arg) {
  job_t* J = (job_t*)arg;
  int64_t ntask = (int64_t)J->nrg * J->sp->ncols;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    int64_t t = J->next_task++;
    pthread_mutex_unlock(&J->mu);
    if (t >= ntask) break;
    /* order tasks column-major so heavy columns of one rg do not serialise */
    int rg = (int)(t % J->nrg), col = (int)(t / J->nrg);
    encode_chunk(J, rg, col);
  }
  return NULL;
}

/* ------------------------------------------------------------------ */
/* file assembly                                                        */
/* ------------------------------------------------------------------ */

static void col_name(int col, char* out) {
  /* "c0", "c1", ... */
  char tmp[16]; int n = 0; int v = col;
  do { tmp[n++] = (char)('0' + v % 10); v /= 10; } while (v);
  out[0] = 'c';
  for (int i = 0; i < n; ++i) out[1 + i] = tmp[n - 1 - i];
  out[1 + n] = 0;
}

/* Writes a whole Parquet file; returns malloc'd bytes (free with pqg_free). */
uint8_t* pqg_write(const pqg_spec* sp, const pqg_col* cols, size_t* out_len) {
  int nrg = sp->num_rows == 0 ? 1 : (int)((sp->num_rows + sp->rg_rows - 1) / sp->rg_rows);
  job_t J;
  memset(&J, 0, sizeof(J));
  J.sp = sp; J.cols = cols; J.nrg = nrg;
  J.gens = (colgen_t*)calloc((size_t)sp->ncols, sizeof(colgen_t));
  for (int c = 0; c < sp->ncols; ++c) colgen_init(&J.gens[c], sp, &cols[c], c);
  J.sorted_base = (int64_t*)calloc((size_t)sp->ncols * (size_t)nrg, sizeof(int64_t));
  for (int c = 0; c < sp->ncols; ++c) {
    if (cols[c].dist != D_SORTED) continue;
    uint64_t k = J.gens[c].start;
    for (int rg = 0; rg < nrg; ++rg) {
      J.sorted_base[(size_t)c * (size_t)nrg + (size_t)rg] = (int64_t)k;
      int64_t r0 = (int64_t)rg * sp->rg_rows;
      int64_t r1 = r0 + sp->rg_rows < sp->num_rows ? r0 + sp->rg_rows : sp->num_rows;
      for (int64_t row = r0; row < r1; ++row) k += sorted_gap(&J.gens[c], row);
    }
  }
  J.outs = (chunk_out_t*)calloc((size_t)nrg * (size_t)sp->ncols, sizeof(chunk_out_t));
  pthread_mutex_init(&J.mu, NULL);
  int nt = sp->nthreads > 0 ? sp->nthreads : 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nt);
  for (int i = 0; i < nt; ++i) pthread_create(&th[i], NULL, worker, &J);
  for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  free(th);
  pthread_mutex_destroy(&J.mu);

  /* total size */
  size_t total = 4;
  for (size_t i = 0; i < (size_t)nrg * (size_t)sp->ncols; ++i) total += J.outs[i].bytes.n;
  buf_t f = {0};
  buf_reserve(&f, total + 4096);
  put_bytes(&f, "PAR1", 4);
  int64_t* base = (int64_t*)malloc(sizeof(int64_t) * (size_t)nrg * (size_t)sp->ncols);
  for (int rg = 0; rg < nrg; ++rg)
    for (int c = 0; c < sp->ncols; ++c) {
      size_t i = (size_t)rg * (size_t)sp->ncols + (size_t)c;
      base[i] = (int64_t)f.n;
      put_bytes(&f, J.outs[i].bytes.p, J.outs[i].bytes.n);
    }
  /* footer */
  size_t foot0 = f.n;
  tw_t t; tw_init(&t, &f);
  tw_i32(&t, 1, sp->page_version == 2 ? 2 : 1);
  tw_list_begin(&t, 2, TT_STRUCT, (size_t)sp->ncols + 1);
  tw_elem_begin(&t);
  tw_bin(&t, 4, "schema", 6);
  tw_i32(&t, 5, sp->ncols);
  tw_elem_end(&t);
  for (int c = 0; c < sp->ncols; ++c) {
    char nm[16]; col_name(c, nm);
    tw_elem_begin(&t);
    tw_i32(&t, 1, cols[c].ptype);
    tw_i32(&t, 3, cols[c].optional ? 1 : 0);
    tw_bin(&t, 4, nm, strlen(nm));
    tw_elem_end(&t);
  }
  tw_i64(&t, 3, sp->num_rows);
  tw_list_begin(&t, 4, TT_STRUCT, (size_t)nrg);
  for (int rg = 0; rg < nrg; ++rg) {
    int64_t r0 = (int64_t)rg * sp->rg_rows;
    int64_t nr = sp->num_rows - r0 < sp->rg_rows ? sp->num_rows - r0 : sp->rg_rows;
    if (nr < 0) nr = 0;
    tw_elem_begin(&t);
    tw_list_begin(&t, 1, TT_STRUCT, (size_t)sp->ncols);
    int64_t rg_bytes = 0;
    for (int c = 0; c < sp->ncols; ++c) {
      size_t i = (size_t)rg * (size_t)sp->ncols + (size_t)c;
      chunk_out_t* co = &J.outs[i];
      char nm[16]; col_name(c, nm);
      rg_bytes += co->uncompressed_total;
      tw_elem_begin(&t);
      tw_i64(&t, 2, base[i] + (int64_t)co->bytes.n);
      tw_struct_begin(&t, 3);
      tw_i32(&t, 1, cols[c].ptype);
      tw_list_begin(&t, 2, TT_I32, (size_t)co->nencs);
      for (int e = 0; e < co->nencs; ++e) put_uleb(&f, zz64(co->encs[e]));
      tw_list_begin(&t, 3, TT_BIN, 1);
      put_uleb(&f, strlen(nm)); put_bytes(&f, nm, strlen(nm));
      tw_i32(&t, 4, co->codec);
      tw_i64(&t, 5, co->num_values);
      tw_i64(&t, 6, co->uncompressed_total);
      tw_i64(&t, 7, (int64_t)co->bytes.n);
      tw_i64(&t, 9, base[i] + co->data_page_rel);
      if (co->dict_page_rel >= 0) tw_i64(&t, 11, base[i] + co->dict_page_rel);
      tw_struct_end(&t);
      tw_elem_end(&t);
    }
    tw_i64(&t, 2, rg_bytes);
    tw_i64(&t, 3, nr);
    tw_elem_end(&t);
  }
  tw_bin(&t, 6, "pqgen", 5);
  put_u8(&f, 0);
  uint32_t flen = (uint32_t)(f.n - foot0);
  put_u32le(&f, flen);
  put_bytes(&f, "PAR1", 4);

  for (size_t i = 0; i < (size_t)nrg * (size_t)sp->ncols; ++i) buf_free(&J.outs[i].bytes);
  free(J.outs);
  free(base);
  free(J.sorted_base);
  for (int c = 0; c < sp->ncols; ++c) colgen_free(&J.gens[c]);
  free(J.gens);
  *out_len = f.n;
  return f.p;
}

void pqg_free(void* p) { free(p); }

/* ------------------------------------------------------------------ */
/* expected decoded columns straight from the generator                 */
/* ------------------------------------------------------------------ */

/* Fixed-width column rows [row0, row0+n): values (zero for nulls) and an
   LSB-first validity bitmap starting at bit 0. */
void pqg_expected_fixed(const pqg_spec* sp, const pqg_col* cols, int col, int64_t row0, int64_t n, void* values, uint8_t* validity) {
  colgen_t g; colgen_init(&g, sp, &cols[col], col);
  const pqg_col* c = &cols[col];
  int w = ptype_width(c->ptype);
  uint64_t key = 0;
  if (c->dist == D_SORTED) { key = g.start; for (int64_t r = 0; r < row0; ++r) key += sorted_gap(&g, r); }
  if (validity) memset(validity, 0, (size_t)((n + 7) / 8));
  for (int64_t i = 0; i < n; ++i) {
    int64_t row = row0 + i;
    int ok = row_valid(&g, row);
    uint64_t x;
    if (c->dist == D_SORTED) { key += sorted_gap(&g, row); x = key; }
    else x = row_value_from_id(&g, row_id(&g, row));
    if (!ok) x = 0;
    memcpy((uint8_t*)values + (size_t)i * (size_t)w, &x, (size_t)w);
    if (ok && validity) validity[i >> 3] |= (uint8_t)(1u << (i & 7));
  }
  colgen_free(&g);
}

/* String column rows [row0, row0+n): offsets[n+1] from 0, chars (may be
   NULL to only size), validity. Returns total chars bytes. */
int64_t pqg_expected_strings(const pqg_spec* sp, const pqg_col* cols, int col, int64_t row0, int64_t n, int64_t* offsets, uint8_t* chars, uint8_t* validity) {
  colgen_t g; colgen_init(&g, sp, &cols[col], col);
  int64_t pos = 0;
  if (validity) memset(validity, 0, (size_t)((n + 7) / 8));
  for (int64_t i = 0; i < n; ++i) {
    int64_t row = row0 + i;
    if (offsets) offsets[i] = pos;
    if (!row_valid(&g, row)) continue;
    uint64_t d = row_id(&g, row);
    int len = string_len(&g, d);
    if (chars) string_fill(&g, d, chars + pos, len);
    pos += len;
    if (validity) validity[i >> 3] |= (uint8_t)(1u << (i & 7));
  }
  if (offsets) offsets[n] = pos;
  colgen_free(&g);
  return pos;
}
