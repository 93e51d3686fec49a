/*
 * oracle.c -- plain, single-threaded CPU Parquet column-chunk reader.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the reference the GPU reader is checked
 * against, bit for bit.  Only tests/, the smoke check and the benchmark's CPU
 * baseline may load it; the GPU product path never calls it.  It shares no
 * code, header or table with the GPU path.
 *
 * What it computes (the plain definition of a Parquet scan): for each
 * selected column and each row of the selected row groups, in row-group,
 * page and value order, the value that was written, or "null" where the
 * definition level is 0.  Output layout: fixed-width values with zeroed null
 * slots, LSB-first validity bits (1 = valid), int64 string offsets starting
 * at 0, and the concatenated string bytes.
 *
 * The paper (Sec. 2) fixes the structure being scanned: a file holds row
 * groups, a row group holds one column chunk per column, a chunk is divided
 * into pages, pages carry V1 or V2 encodings, and compression (here Snappy)
 * applies per chunk.  Sec. 3 (Encoding Flexibility) names the encodings
 * decoded here: PLAIN, dictionary (V1) and DELTA_BINARY_PACKED (V2), and
 * asks for every valid Parquet encoding of a type to be a candidate, which
 * adds DELTA_LENGTH_BYTE_ARRAY and DELTA_BYTE_ARRAY for strings and
 * BYTE_STREAM_SPLIT for fixed-width values.  The byte-level rules come from
 * the public Apache Parquet format description (Thrift compact footer and
 * page headers, RLE/bit-packed hybrid, DELTA_BINARY_PACKED, the string delta
 * encodings, BYTE_STREAM_SPLIT, PLAIN) and the public Snappy raw-format
 * description.
 *
 * Everything is deliberately slow and literal: bits are read one at a time,
 * every length is checked before it is used, and no step is fused.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ECORRUPT -2
#define ORC_EUNSUPPORTED -3
#define ORC_ENOMEM -4

static char g_err[256];
static int fail(int code, const char* msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg);
  return code;
}
const char* orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ */
/* bounded byte reader                                                  */
/* ------------------------------------------------------------------ */

typedef struct {
  const uint8_t* p;
  uint64_t n;
  uint64_t pos;
  int bad;
} rd_t;

static int rd_byte(rd_t* r, uint8_t* out) {
  if (r->pos >= r->n) { r->bad = 1; return 0; }
  *out = r->p[r->pos++];
  return 1;
}

/* unsigned LEB128, at most 10 bytes */
static uint64_t rd_uleb(rd_t* r) {
  uint64_t v = 0;
  for (int shift = 0; shift < 70; shift += 7) {
    uint8_t b;
    if (!rd_byte(r, &b)) return 0;
    if (shift == 63 && (b & 0x7e)) { r->bad = 1; return 0; }
    v |= (uint64_t)(b & 0x7f) << shift;
    if (!(b & 0x80)) return v;
  }
  r->bad = 1;
  return 0;
}
static int64_t unzigzag(uint64_t v) { return (int64_t)(v >> 1) ^ -(int64_t)(v & 1); }

/* ------------------------------------------------------------------ */
/* Thrift compact protocol (decode side)                                */
/* ------------------------------------------------------------------ */

enum { T_STOP = 0, T_TRUE = 1, T_FALSE = 2, T_I8 = 3, T_I16 = 4, T_I32 = 5, T_I64 = 6, T_DOUBLE = 7,
       T_BINARY = 8, T_LIST = 9, T_SET = 10, T_MAP = 11, T_STRUCT = 12 };

/* Reads the next field header of a struct.  Returns 0 at STOP. */
static int th_field(rd_t* r, int* last_id, int* id, int* type) {
  uint8_t b;
  if (!rd_byte(r, &b)) return 0;
  if (b == 0) return 0;
  *type = b & 0x0f;
  int delta = b >> 4;
  if (delta) *id = *last_id + delta;
  else *id = (int)unzigzag(rd_uleb(r));
  *last_id = *id;
  return !r->bad;
}

static void th_skip(rd_t* r, int type, int depth);

static void th_skip_struct(rd_t* r, int depth) {
  int last = 0, id, type;
  while (!r->bad && th_field(r, &last, &id, &type)) th_skip(r, type, depth + 1);
}

static void th_list_header(rd_t* r, uint64_t* n, int* etype) {
  uint8_t b;
  if (!rd_byte(r, &b)) return;
  *etype = b & 0x0f;
  uint64_t sz = b >> 4;
  if (sz == 15) sz = rd_uleb(r);
  *n = sz;
}

static void th_skip(rd_t* r, int type, int depth) {
  if (depth > 64) { r->bad = 1; return; }
  uint8_t b;
  switch (type) {
    case T_TRUE: case T_FALSE: return;
    case T_I8: rd_byte(r, &b); return;
    case T_I16: case T_I32: case T_I64: rd_uleb(r); return;
    case T_DOUBLE: if (r->pos + 8 > r->n) r->bad = 1; else r->pos += 8; return;
    case T_BINARY: {
      uint64_t len = rd_uleb(r);
      if (r->bad || len > r->n - r->pos) { r->bad = 1; return; }
      r->pos += len;
      return;
    }
    case T_LIST: case T_SET: {
      uint64_t n = 0; int et = 0;
      th_list_header(r, &n, &et);
      for (uint64_t i = 0; i < n && !r->bad; ++i) {
        if (et == T_TRUE || et == T_FALSE) rd_byte(r, &b); /* bool elements are one byte */
        else th_skip(r, et, depth + 1);
      }
      return;
    }
    case T_MAP: {
      uint64_t n = rd_uleb(r);
      if (n == 0) return;
      uint8_t kv;
      if (!rd_byte(r, &kv)) return;
      for (uint64_t i = 0; i < n && !r->bad; ++i) { th_skip(r, kv >> 4, depth + 1); th_skip(r, kv & 15, depth + 1); }
      return;
    }
    case T_STRUCT: th_skip_struct(r, depth); return;
    default: r->bad = 1; return;
  }
}

static int64_t th_int(rd_t* r) { return unzigzag(rd_uleb(r)); }

/* ------------------------------------------------------------------ */
/* footer model                                                         */
/* ------------------------------------------------------------------ */

typedef struct {
  int type, optional;
  char name[64];
} orc_schema_col;

typedef struct {
  int type, codec;
  int64_t num_values, total_compressed, data_page_offset, dict_page_offset;
  int has_dict_offset;
} orc_chunk;

struct orc_file {
  const uint8_t* buf;
  uint64_t len;
  int ncols, nrg;
  orc_schema_col* cols;
  int64_t* rg_rows;
  orc_chunk* chunks; /* [rg][col] */
};
typedef struct orc_file orc_file;

static int parse_schema_element(rd_t* r, int* type, int* rep, int* nchildren, char* name) {
  int last = 0, id, t;
  *type = -1; *rep = 0; *nchildren = 0; name[0] = 0;
  while (th_field(r, &last, &id, &t)) {
    if (id == 1 && t == T_I32) *type = (int)th_int(r);
    else if (id == 3 && t == T_I32) *rep = (int)th_int(r);
    else if (id == 5 && t == T_I32) *nchildren = (int)th_int(r);
    else if (id == 4 && t == T_BINARY) {
      uint64_t len = rd_uleb(r);
      if (r->bad || len > r->n - r->pos) { r->bad = 1; return 0; }
      uint64_t k = len < 63 ? len : 63;
      memcpy(name, r->p + r->pos, k);
      name[k] = 0;
      r->pos += len;
    } else th_skip(r, t, 1);
  }
  return !r->bad;
}

static int parse_column_meta(rd_t* r, orc_chunk* c) {
  int last = 0, id, t;
  c->has_dict_offset = 0;
  c->codec = 0;
  while (th_field(r, &last, &id, &t)) {
    if (id == 1 && t == T_I32) c->type = (int)th_int(r);
    else if (id == 4 && t == T_I32) c->codec = (int)th_int(r);
    else if (id == 5 && t == T_I64) c->num_values = th_int(r);
    else if (id == 7 && t == T_I64) c->total_compressed = th_int(r);
    else if (id == 9 && t == T_I64) c->data_page_offset = th_int(r);
    else if (id == 11 && t == T_I64) { c->dict_page_offset = th_int(r); c->has_dict_offset = 1; }
    else th_skip(r, t, 1);
  }
  return !r->bad;
}

static int parse_column_chunk(rd_t* r, orc_chunk* c) {
  int last = 0, id, t, got = 0;
  while (th_field(r, &last, &id, &t)) {
    if (id == 3 && t == T_STRUCT) { if (!parse_column_meta(r, c)) return 0; got = 1; }
    else if (id == 1 && t == T_BINARY) { th_skip(r, t, 1); r->bad = r->bad ? 1 : 2; } /* external file */
    else th_skip(r, t, 1);
  }
  return got && r->bad == 0;
}

void orc_close(orc_file* f) {
  if (!f) return;
  free(f->cols); free(f->rg_rows); free(f->chunks); free(f);
}

/* File check and footer decode (format: "PAR1", chunks, footer, u32 LE
   footer length, "PAR1"). */
int orc_open(const uint8_t* buf, uint64_t len, orc_file** out) {
  *out = NULL;
  if (!buf) return fail(ORC_EINVAL, "null buffer");
  if (len < 12) return fail(ORC_ECORRUPT, "file shorter than 12 bytes");
  if (memcmp(buf, "PAR1", 4) || memcmp(buf + len - 4, "PAR1", 4)) return fail(ORC_ECORRUPT, "bad magic");
  uint64_t flen = (uint64_t)buf[len - 8] | ((uint64_t)buf[len - 7] << 8) | ((uint64_t)buf[len - 6] << 16) | ((uint64_t)buf[len - 5] << 24);
  if (flen + 12 > len) return fail(ORC_ECORRUPT, "footer length exceeds file");
  rd_t r = {buf + len - 8 - flen, flen, 0, 0};
  orc_file* f = (orc_file*)calloc(1, sizeof(orc_file));
  f->buf = buf; f->len = len;
  int last = 0, id, t;
  int have_schema = 0, have_rgs = 0;
  while (th_field(&r, &last, &id, &t)) {
    if (id == 2 && t == T_LIST) {
      uint64_t n = 0; int et = 0;
      th_list_header(&r, &n, &et);
      if (r.bad || et != T_STRUCT || n < 1 || n > 100000) { orc_close(f); return fail(ORC_ECORRUPT, "bad schema list"); }
      int type, rep, nch; char name[64];
      if (!parse_schema_element(&r, &type, &rep, &nch, name)) { orc_close(f); return fail(ORC_ECORRUPT, "bad root schema"); }
      if ((uint64_t)nch != n - 1) { orc_close(f); return fail(ORC_EUNSUPPORTED, "nested schema"); }
      f->ncols = nch;
      f->cols = (orc_schema_col*)calloc((size_t)(nch > 0 ? nch : 1), sizeof(orc_schema_col));
      for (int c = 0; c < f->ncols; ++c) {
        int leaf_children = 0;
        if (!parse_schema_element(&r, &type, &rep, &leaf_children, name)) { orc_close(f); return fail(ORC_ECORRUPT, "bad schema element"); }
        if (leaf_children != 0 || type < 0) { orc_close(f); return fail(ORC_EUNSUPPORTED, "nested schema"); }
        if (rep == 2) { orc_close(f); return fail(ORC_EUNSUPPORTED, "repeated column"); }
        if (type != 1 && type != 2 && type != 5 && type != 6) { orc_close(f); return fail(ORC_EUNSUPPORTED, "unsupported physical type"); }
        f->cols[c].type = type;
        f->cols[c].optional = rep == 1;
        memcpy(f->cols[c].name, name, 64);
      }
      have_schema = 1;
    } else if (id == 4 && t == T_LIST) {
      uint64_t n = 0; int et = 0;
      th_list_header(&r, &n, &et);
      if (r.bad || et != T_STRUCT || !have_schema || n > 10000000) { orc_close(f); return fail(ORC_ECORRUPT, "bad row group list"); }
      f->nrg = (int)n;
      f->rg_rows = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
      f->chunks = (orc_chunk*)calloc((size_t)(n > 0 ? n : 1) * (size_t)(f->ncols > 0 ? f->ncols : 1), sizeof(orc_chunk));
      for (uint64_t g = 0; g < n; ++g) {
        int l2 = 0, id2, t2, ncc = 0;
        while (th_field(&r, &l2, &id2, &t2)) {
          if (id2 == 1 && t2 == T_LIST) {
            uint64_t m = 0; int e2 = 0;
            th_list_header(&r, &m, &e2);
            if (r.bad || e2 != T_STRUCT || m != (uint64_t)f->ncols) { orc_close(f); return fail(ORC_ECORRUPT, "column count mismatch"); }
            for (uint64_t c = 0; c < m; ++c)
              if (!parse_column_chunk(&r, &f->chunks[g * (uint64_t)f->ncols + c])) { orc_close(f); return fail(r.bad == 2 ? ORC_EUNSUPPORTED : ORC_ECORRUPT, "bad column chunk"); }
            ncc = 1;
          } else if (id2 == 3 && t2 == T_I64) f->rg_rows[g] = th_int(&r);
          else th_skip(&r, t2, 1);
        }
        if (!ncc && f->ncols > 0) { orc_close(f); return fail(ORC_ECORRUPT, "row group without columns"); }
      }
      have_rgs = 1;
    } else th_skip(&r, t, 0);
    if (r.bad) break;
  }
  if (r.bad || !have_schema || !have_rgs) { orc_close(f); return fail(ORC_ECORRUPT, "bad footer"); }
  for (int g = 0; g < f->nrg; ++g)
    for (int c = 0; c < f->ncols; ++c) {
      orc_chunk* ch = &f->chunks[(size_t)g * (size_t)f->ncols + (size_t)c];
      if (ch->type != f->cols[c].type) { orc_close(f); return fail(ORC_ECORRUPT, "chunk type differs from schema"); }
      if (ch->codec != 0 && ch->codec != 1) { orc_close(f); return fail(ORC_EUNSUPPORTED, "codec other than UNCOMPRESSED/SNAPPY"); }
      if (f->rg_rows[g] < 0 || ch->num_values != f->rg_rows[g]) { orc_close(f); return fail(ORC_ECORRUPT, "chunk value count differs from row group rows"); }
    }
  *out = f;
  return ORC_OK;
}

int orc_num_columns(const orc_file* f) { return f->ncols; }
int orc_num_row_groups(const orc_file* f) { return f->nrg; }
int64_t orc_row_group_rows(const orc_file* f, int rg) { return f->rg_rows[rg]; }
int orc_column_type(const orc_file* f, int c) { return f->cols[c].type; }
int orc_column_optional(const orc_file* f, int c) { return f->cols[c].optional; }

/* ------------------------------------------------------------------ */
/* page header                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
  int32_t type, uncompressed_size, compressed_size;
  int32_t num_values, encoding;       /* V1 data, dictionary, V2 */
  int32_t num_nulls, num_rows;        /* V2 */
  int32_t def_len, rep_len;           /* V2 */
  int32_t is_compressed;              /* V2, default 1 */
  int32_t has_sub;                    /* the type-specific header was present */
} orc_page_header;

static int parse_data_header(rd_t* r, orc_page_header* h, int v2) {
  int last = 0, id, t;
  while (th_field(r, &last, &id, &t)) {
    if (t == T_TRUE || t == T_FALSE) { if (v2 && id == 7) h->is_compressed = (t == T_TRUE); continue; }
    if (id == 1 && t == T_I32) h->num_values = (int32_t)th_int(r);
    else if (!v2 && id == 2 && t == T_I32) h->encoding = (int32_t)th_int(r);
    else if (v2 && id == 2 && t == T_I32) h->num_nulls = (int32_t)th_int(r);
    else if (v2 && id == 3 && t == T_I32) h->num_rows = (int32_t)th_int(r);
    else if (v2 && id == 4 && t == T_I32) h->encoding = (int32_t)th_int(r);
    else if (v2 && id == 5 && t == T_I32) h->def_len = (int32_t)th_int(r);
    else if (v2 && id == 6 && t == T_I32) h->rep_len = (int32_t)th_int(r);
    else th_skip(r, t, 2);
  }
  h->has_sub = 1;
  return !r->bad;
}

/* Decodes one PageHeader; returns its length in bytes, or a negative code. */
int64_t orc_page_header_parse(const uint8_t* p, uint64_t n, orc_page_header* h) {
  memset(h, 0, sizeof(*h));
  h->type = -1;
  h->is_compressed = 1;
  rd_t r = {p, n, 0, 0};
  int last = 0, id, t;
  while (th_field(&r, &last, &id, &t)) {
    if (id == 1 && t == T_I32) h->type = (int32_t)th_int(&r);
    else if (id == 2 && t == T_I32) h->uncompressed_size = (int32_t)th_int(&r);
    else if (id == 3 && t == T_I32) h->compressed_size = (int32_t)th_int(&r);
    else if (id == 5 && t == T_STRUCT) parse_data_header(&r, h, 0);
    else if (id == 7 && t == T_STRUCT) parse_data_header(&r, h, 0);
    else if (id == 8 && t == T_STRUCT) parse_data_header(&r, h, 1);
    else th_skip(&r, t, 1);
    if (r.bad) break;
  }
  if (r.bad) return ORC_ECORRUPT;
  if (h->uncompressed_size < 0 || h->compressed_size < 0) return ORC_ECORRUPT;
  return (int64_t)r.pos;
}

/* ------------------------------------------------------------------ */
/* Snappy raw format                                                    */
/* ------------------------------------------------------------------ */

/* Decompresses a whole Snappy stream into dst[0..cap).  Returns the
   decompressed length or a negative code. */
int64_t orc_snappy_decompress(const uint8_t* src, uint64_t n, uint8_t* dst, uint64_t cap) {
  rd_t r = {src, n, 0, 0};
  uint64_t total = rd_uleb(&r);
  if (r.bad || total > 0xffffffffull) return ORC_ECORRUPT;
  if (total > cap) return ORC_ECORRUPT;
  uint64_t op = 0;
  while (r.pos < n) {
    uint8_t t = src[r.pos++];
    uint64_t len, off;
    if ((t & 3) == 0) {
      uint64_t l = t >> 2;
      if (l >= 60) {
        uint64_t nb = l - 59;
        if (r.pos + nb > n) return ORC_ECORRUPT;
        l = 0;
        for (uint64_t k = 0; k < nb; ++k) l |= (uint64_t)src[r.pos + k] << (8 * k);
        r.pos += nb;
      }
      len = l + 1;
      if (r.pos + len > n || op + len > total) return ORC_ECORRUPT;
      for (uint64_t k = 0; k < len; ++k) dst[op + k] = src[r.pos + k];
      r.pos += len;
      op += len;
      continue;
    }
    if ((t & 3) == 1) {
      if (r.pos + 1 > n) return ORC_ECORRUPT;
      len = 4 + ((t >> 2) & 7);
      off = ((uint64_t)(t >> 5) << 8) | src[r.pos];
      r.pos += 1;
    } else if ((t & 3) == 2) {
      if (r.pos + 2 > n) return ORC_ECORRUPT;
      len = (uint64_t)(t >> 2) + 1;
      off = (uint64_t)src[r.pos] | ((uint64_t)src[r.pos + 1] << 8);
      r.pos += 2;
    } else {
      if (r.pos + 4 > n) return ORC_ECORRUPT;
      len = (uint64_t)(t >> 2) + 1;
      off = (uint64_t)src[r.pos] | ((uint64_t)src[r.pos + 1] << 8) | ((uint64_t)src[r.pos + 2] << 16) | ((uint64_t)src[r.pos + 3] << 24);
      r.pos += 4;
    }
    if (off == 0 || off > op || op + len > total) return ORC_ECORRUPT;
    for (uint64_t k = 0; k < len; ++k) dst[op + k] = dst[op + k - off]; /* forward, byte by byte */
    op += len;
  }
  if (op != total) return ORC_ECORRUPT;
  return (int64_t)op;
}

/* ------------------------------------------------------------------ */
/* bit reading, RLE/bit-packed hybrid                                   */
/* ------------------------------------------------------------------ */

/* w bits starting at bit position `bit` of p, least significant bit first */
static uint64_t get_bits(const uint8_t* p, uint64_t bit, int w) {
  uint64_t v = 0;
  for (int j = 0; j < w; ++j) {
    uint64_t b = bit + (uint64_t)j;
    v |= (uint64_t)((p[b >> 3] >> (b & 7)) & 1) << j;
  }
  return v;
}

/* Decodes `count` values of width w from an RLE/bit-packed hybrid stream
   p[0..n).  A header h with h&1 announces (h>>1) groups of 8 bit-packed
   values in (h>>1)*w bytes; otherwise an RLE run of (h>>1) copies of a
   ceil(w/8)-byte little-endian value.  Values past `count` are dropped.
   Returns the bytes consumed, or a negative code if the stream ends early. */
int64_t orc_hybrid_decode(const uint8_t* p, uint64_t n, int w, int64_t count, uint32_t* out) {
  if (w < 0 || w > 32) return ORC_ECORRUPT;
  rd_t r = {p, n, 0, 0};
  int64_t k = 0;
  while (k < count) {
    uint64_t h = rd_uleb(&r);
    if (r.bad) return ORC_ECORRUPT;
    if (h & 1) {
      uint64_t groups = h >> 1;
      uint64_t nbytes = groups * (uint64_t)w;
      if (groups > (1ull << 40) || nbytes > n - r.pos) return ORC_ECORRUPT;
      for (uint64_t i = 0; i < groups * 8; ++i) {
        if (k >= count) break;
        out[k++] = (uint32_t)get_bits(p + r.pos, i * (uint64_t)w, w);
      }
      r.pos += nbytes;
    } else {
      uint64_t run = h >> 1;
      uint64_t vb = (uint64_t)(w + 7) / 8;
      if (vb > n - r.pos) return ORC_ECORRUPT;
      uint64_t v = 0;
      for (uint64_t j = 0; j < vb; ++j) v |= (uint64_t)p[r.pos + j] << (8 * j);
      r.pos += vb;
      for (uint64_t i = 0; i < run && k < count; ++i) out[k++] = (uint32_t)v;
    }
  }
  return (int64_t)r.pos;
}

/* ------------------------------------------------------------------ */
/* DELTA_BINARY_PACKED                                                  */
/* ------------------------------------------------------------------ */

/* Header: block size, miniblocks per block, total count, zigzag first
   value.  Each block: zigzag min delta, one bit-width byte per miniblock,
   then the miniblock bodies; v[i] = v[i-1] + min_delta + packed[i], with
   wrap-around at the physical width.  Bodies of miniblocks after the last
   value are absent.  Returns bytes consumed or a negative code. */
int64_t orc_delta_decode(const uint8_t* p, uint64_t n, int is32, int64_t count, uint64_t* out) {
  rd_t r = {p, n, 0, 0};
  uint64_t block = rd_uleb(&r), mini = rd_uleb(&r), total = rd_uleb(&r);
  int64_t first = unzigzag(rd_uleb(&r));
  if (r.bad) return ORC_ECORRUPT;
  if (block == 0 || block % 128 != 0 || mini == 0 || block % mini != 0 || (block / mini) % 32 != 0) return ORC_ECORRUPT;
  if ((int64_t)total != count) return ORC_ECORRUPT;
  if (total == 0) return (int64_t)r.pos;
  uint64_t per = block / mini;
  uint64_t prev = is32 ? (uint64_t)(uint32_t)first : (uint64_t)first;
  out[0] = prev;
  uint64_t k = 1;
  while (k < total) {
    int64_t min_delta = unzigzag(rd_uleb(&r));
    if (r.bad || mini > n - r.pos) return ORC_ECORRUPT;
    const uint8_t* widths = p + r.pos;
    r.pos += mini;
    for (uint64_t m = 0; m < mini && k < total; ++m) {
      int w = widths[m];
      if (w > (is32 ? 32 : 64)) return ORC_ECORRUPT;
      uint64_t nbytes = per * (uint64_t)w / 8;
      if (nbytes > n - r.pos) return ORC_ECORRUPT;
      for (uint64_t i = 0; i < per && k < total; ++i) {
        uint64_t u = get_bits(p + r.pos, i * (uint64_t)w, w);
        prev = prev + (uint64_t)min_delta + u;
        if (is32) prev = (uint64_t)(uint32_t)prev;
        out[k++] = prev;
      }
      r.pos += nbytes;
    }
  }
  return (int64_t)r.pos;
}

/* ------------------------------------------------------------------ */
/* BYTE_STREAM_SPLIT                                                    */
/* ------------------------------------------------------------------ */

/* The page's `count` values of `w` bytes are stored as w streams of
   `count` bytes each: stream b holds byte b (little-endian position) of
   every value, so value k's byte b is p[b * count + k].  Returns the bytes
   used or a negative code. */
int64_t orc_byte_stream_split_decode(const uint8_t* p, uint64_t n, int w, int64_t count, uint64_t* out) {
  if (w < 1 || w > 8 || count < 0) return ORC_EINVAL;
  if ((uint64_t)count * (uint64_t)w > n) return ORC_ECORRUPT;
  for (int64_t k = 0; k < count; ++k) {
    uint64_t v = 0;
    for (int b = 0; b < w; ++b) v |= (uint64_t)p[(uint64_t)b * (uint64_t)count + (uint64_t)k] << (8 * b);
    out[k] = v;
  }
  return count * w;
}

/* ------------------------------------------------------------------ */
/* DELTA_LENGTH_BYTE_ARRAY and DELTA_BYTE_ARRAY                         */
/* ------------------------------------------------------------------ */

/* DELTA_LENGTH_BYTE_ARRAY: the `count` lengths as one DELTA_BINARY_PACKED
   stream of 32-bit values, then all the strings' bytes back to back.  Gives
   each string's position (from p) and length; a negative length or bytes
   past the stream are corrupt.  Returns the bytes used. */
int64_t orc_delta_length_decode(const uint8_t* p, uint64_t n, int64_t count, uint64_t* pos, uint32_t* len) {
  uint64_t* lens = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(count > 0 ? count : 1));
  if (!lens) return ORC_ENOMEM;
  int64_t used = orc_delta_decode(p, n, 1, count, lens);
  if (used < 0) { free(lens); return used; }
  uint64_t q = (uint64_t)used;
  for (int64_t k = 0; k < count; ++k) {
    int32_t l = (int32_t)(uint32_t)lens[k];
    if (l < 0 || (uint64_t)l > n - q) { free(lens); return ORC_ECORRUPT; }
    pos[k] = q;
    len[k] = (uint32_t)l;
    q += (uint64_t)l;
  }
  free(lens);
  return (int64_t)q;
}

/* DELTA_BYTE_ARRAY: the `count` prefix lengths as a DELTA_BINARY_PACKED
   stream of 32-bit values, then the suffixes as DELTA_LENGTH_BYTE_ARRAY.
   String k is the first prefix[k] bytes of string k-1 followed by suffix k
   (string 0 has no predecessor: its prefix length must be 0; every prefix
   length must lie in [0, length of the previous string]).  The strings are
   written one after the other into *mat (grown with realloc, *mat_cap bytes
   allocated), with their positions in *mat and lengths.  Returns the bytes
   used. */
int64_t orc_delta_byte_array_decode(const uint8_t* p, uint64_t n, int64_t count, uint8_t** mat, uint64_t* mat_cap,
                                    uint64_t* pos, uint32_t* len) {
  size_t m = (size_t)(count > 0 ? count : 1);
  uint64_t* pre = (uint64_t*)malloc(sizeof(uint64_t) * m);
  uint64_t* spos = (uint64_t*)malloc(sizeof(uint64_t) * m);
  uint32_t* slen = (uint32_t*)malloc(sizeof(uint32_t) * m);
  int64_t rc = ORC_OK;
  if (!pre || !spos || !slen) { rc = ORC_ENOMEM; goto done; }
  int64_t used = orc_delta_decode(p, n, 1, count, pre);
  if (used < 0) { rc = used; goto done; }
  int64_t used2 = orc_delta_length_decode(p + used, n - (uint64_t)used, count, spos, slen);
  if (used2 < 0) { rc = used2; goto done; }
  uint64_t at = 0;
  for (int64_t k = 0; k < count; ++k) {
    int32_t pk = (int32_t)(uint32_t)pre[k];
    uint64_t prev_len = k > 0 ? len[k - 1] : 0;
    if (pk < 0 || (uint64_t)pk > prev_len) { rc = ORC_ECORRUPT; goto done; }
    uint64_t total = (uint64_t)pk + slen[k];
    if (total > 0xffffffffull) { rc = ORC_ECORRUPT; goto done; }
    if (at + total > *mat_cap) {
      uint64_t cap = (*mat_cap ? *mat_cap : 1024);
      while (cap < at + total) cap *= 2;
      uint8_t* nm = (uint8_t*)realloc(*mat, (size_t)cap);
      if (!nm) { rc = ORC_ENOMEM; goto done; }
      *mat = nm;
      *mat_cap = cap;
    }
    /* the prefix from the previous string, then the suffix */
    for (uint64_t j = 0; j < (uint64_t)pk; ++j) (*mat)[at + j] = (*mat)[pos[k - 1] + j];
    for (uint64_t j = 0; j < slen[k]; ++j) (*mat)[at + (uint64_t)pk + j] = p[(uint64_t)used + spos[k] + j];
    pos[k] = at;
    len[k] = (uint32_t)total;
    at += total;
  }
  rc = used + used2;
done:
  free(pre); free(spos); free(slen);
  return rc;
}

/* ------------------------------------------------------------------ */
/* column read                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t rows;
  void* values;        /* rows * width (fixed-width columns) */
  uint8_t* validity;   /* (rows+7)/8 */
  int64_t* offsets;    /* rows+1 (BYTE_ARRAY) */
  uint8_t* chars;
  int64_t chars_len;
  int64_t pages;       /* data pages read */
  int64_t dict_pages;
} orc_column;

void orc_column_free(orc_column* c) {
  free(c->values); free(c->validity); free(c->offsets); free(c->chars);
  memset(c, 0, sizeof(*c));
}

typedef struct {
  /* dictionary: fixed-width entries as u64, or string (pos,len) into dict_body */
  int64_t n;
  uint64_t* fixed;
  uint64_t* spos;
  uint32_t* slen;
  uint8_t* body; /* owned copy of the (decompressed) dictionary page */
} orc_dict;

static void dict_clear(orc_dict* d) { free(d->fixed); free(d->spos); free(d->slen); free(d->body); memset(d, 0, sizeof(*d)); }

static int width_of(int type) { return type == 1 ? 4 : 8; }

static int chars_append(orc_column* out, int64_t* cap, const uint8_t* s, uint64_t len) {
  if (out->chars_len + (int64_t)len > *cap) {
    int64_t nc = *cap ? *cap : 4096;
    while (nc < out->chars_len + (int64_t)len) nc *= 2;
    uint8_t* np_ = (uint8_t*)realloc(out->chars, (size_t)nc);
    if (!np_) return 0;
    out->chars = np_;
    *cap = nc;
  }
  memcpy(out->chars + out->chars_len, s, len);
  out->chars_len += (int64_t)len;
  return 1;
}

/* Reads column `col` over row groups [rg_b, rg_e) into freshly allocated
   buffers. */
int orc_read_column(orc_file* f, int col, int rg_b, int rg_e, orc_column* out) {
  memset(out, 0, sizeof(*out));
  if (!f || col < 0 || col >= f->ncols || rg_b < 0 || rg_e > f->nrg || rg_b > rg_e) return fail(ORC_EINVAL, "bad column or row-group range");
  int type = f->cols[col].type, optional = f->cols[col].optional;
  int64_t rows = 0;
  for (int g = rg_b; g < rg_e; ++g) rows += f->rg_rows[g];
  out->rows = rows;
  out->validity = (uint8_t*)calloc((size_t)((rows + 7) / 8 + 1), 1);
  int64_t chars_cap = 0;
  if (type == 6) out->offsets = (int64_t*)calloc((size_t)rows + 1, sizeof(int64_t));
  else out->values = calloc((size_t)(rows > 0 ? rows : 1), (size_t)width_of(type));
  if (!out->validity || (type == 6 ? !out->offsets : !out->values)) return fail(ORC_ENOMEM, "out of memory");

  int64_t row = 0; /* output row of the next page's first row */
  int rc = ORC_OK;
  uint32_t* defs = NULL;
  uint32_t* idx = NULL;
  uint64_t* dvals = NULL;
  uint8_t* body = NULL;
  uint8_t* mat = NULL;    /* DELTA_BYTE_ARRAY strings, materialised */
  uint64_t mat_cap = 0;
  orc_dict dict;
  memset(&dict, 0, sizeof(dict));

  for (int g = rg_b; g < rg_e && rc == ORC_OK; ++g) {
    orc_chunk* ch = &f->chunks[(size_t)g * (size_t)f->ncols + (size_t)col];
    dict_clear(&dict);
    int have_dict = 0;
    /* chunk bounds */
    int64_t start = ch->data_page_offset;
    if (ch->has_dict_offset && ch->dict_page_offset > 0 && ch->dict_page_offset < ch->data_page_offset) start = ch->dict_page_offset;
    int64_t end = start + ch->total_compressed;
    if (start < 4 || ch->total_compressed < 0 || end > (int64_t)f->len - 8) { rc = fail(ORC_ECORRUPT, "chunk outside file"); break; }
    int64_t pos = start;
    int64_t chunk_rows = 0;
    int first_page = 1;
    while (pos < end) {
      orc_page_header h;
      int64_t hl = orc_page_header_parse(f->buf + pos, (uint64_t)(end - pos), &h);
      if (hl < 0) { rc = fail(ORC_ECORRUPT, "bad page header"); break; }
      int64_t pay = pos + hl;
      if (h.compressed_size > end - pay) { rc = fail(ORC_ECORRUPT, "page payload overruns chunk"); break; }
      pos = pay + h.compressed_size;
      const uint8_t* payload = f->buf + pay;
      if (h.type == 2) { /* dictionary page */
        if (!first_page || have_dict) { rc = fail(ORC_ECORRUPT, "dictionary page not first"); break; }
        if (!h.has_sub) { rc = fail(ORC_ECORRUPT, "dictionary page without header"); break; }
        if (h.encoding != 0 && h.encoding != 2) { rc = fail(ORC_EUNSUPPORTED, "dictionary encoding"); break; }
        if (h.num_values < 0) { rc = fail(ORC_ECORRUPT, "negative dictionary size"); break; }
        dict.body = (uint8_t*)malloc((size_t)h.uncompressed_size + 1);
        if (ch->codec == 1) {
          int64_t got = orc_snappy_decompress(payload, (uint64_t)h.compressed_size, dict.body, (uint64_t)h.uncompressed_size);
          if (got != h.uncompressed_size) { rc = fail(ORC_ECORRUPT, "dictionary page decompression"); break; }
        } else {
          if (h.compressed_size != h.uncompressed_size) { rc = fail(ORC_ECORRUPT, "dictionary page sizes differ"); break; }
          memcpy(dict.body, payload, (size_t)h.uncompressed_size);
        }
        dict.n = h.num_values;
        uint64_t blen = (uint64_t)h.uncompressed_size;
        if (type == 6) {
          dict.spos = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(dict.n + 1));
          dict.slen = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(dict.n + 1));
          uint64_t q = 0;
          for (int64_t k = 0; k < dict.n; ++k) {
            if (blen - q < 4) { rc = fail(ORC_ECORRUPT, "dictionary string length truncated"); break; }
            uint32_t l = (uint32_t)dict.body[q] | ((uint32_t)dict.body[q + 1] << 8) | ((uint32_t)dict.body[q + 2] << 16) | ((uint32_t)dict.body[q + 3] << 24);
            q += 4;
            if (l > blen - q) { rc = fail(ORC_ECORRUPT, "dictionary string truncated"); break; }
            dict.spos[k] = q; dict.slen[k] = l;
            q += l;
          }
        } else {
          uint64_t w = (uint64_t)width_of(type);
          if ((uint64_t)dict.n * w > blen) { rc = fail(ORC_ECORRUPT, "dictionary page too short"); break; }
          dict.fixed = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(dict.n + 1));
          for (int64_t k = 0; k < dict.n; ++k) {
            uint64_t v = 0;
            for (uint64_t j = 0; j < w; ++j) v |= (uint64_t)dict.body[(uint64_t)k * w + j] << (8 * j);
            dict.fixed[k] = v;
          }
        }
        if (rc != ORC_OK) break;
        have_dict = 1;
        out->dict_pages++;
        first_page = 0;
        continue;
      }
      first_page = 0;
      if (h.type != 0 && h.type != 3) continue; /* index pages and unknown types are skipped */
      if (!h.has_sub) { rc = fail(ORC_ECORRUPT, "data page without header"); break; }
      int64_t nv = h.num_values;
      if (nv < 0 || chunk_rows + nv > f->rg_rows[g]) { rc = fail(ORC_ECORRUPT, "page value count exceeds row group"); break; }

      /* page body: levels and values */
      const uint8_t* lv = NULL; uint64_t lv_len = 0;      /* definition levels */
      const uint8_t* vals = NULL; uint64_t vals_len = 0;  /* encoded values */
      free(body); body = NULL;
      if (h.type == 0) {
        uint64_t blen = (uint64_t)h.uncompressed_size;
        body = (uint8_t*)malloc((size_t)blen + 1);
        if (ch->codec == 1) {
          int64_t got = orc_snappy_decompress(payload, (uint64_t)h.compressed_size, body, blen);
          if (got < 0 || (uint64_t)got != blen) { rc = fail(ORC_ECORRUPT, "data page decompression"); break; }
        } else {
          if (h.compressed_size != h.uncompressed_size) { rc = fail(ORC_ECORRUPT, "data page sizes differ"); break; }
          memcpy(body, payload, (size_t)blen);
        }
        uint64_t q = 0;
        if (optional) {
          if (blen < 4) { rc = fail(ORC_ECORRUPT, "missing level length"); break; }
          uint64_t L = (uint64_t)body[0] | ((uint64_t)body[1] << 8) | ((uint64_t)body[2] << 16) | ((uint64_t)body[3] << 24);
          if (L > blen - 4) { rc = fail(ORC_ECORRUPT, "level length exceeds page"); break; }
          lv = body + 4; lv_len = L;
          q = 4 + L;
        }
        vals = body + q; vals_len = blen - q;
      } else { /* DATA_PAGE_V2 */
        if (h.def_len < 0 || h.rep_len < 0 || (int64_t)h.def_len + h.rep_len > h.compressed_size || h.def_len + h.rep_len > h.uncompressed_size) { rc = fail(ORC_ECORRUPT, "bad V2 level lengths"); break; }
        if (h.rep_len != 0) { rc = fail(ORC_EUNSUPPORTED, "repetition levels"); break; }
        if (h.num_rows != h.num_values) { rc = fail(ORC_ECORRUPT, "V2 rows differ from values"); break; }
        if (!optional && h.def_len != 0) { rc = fail(ORC_ECORRUPT, "levels on a required column"); break; }
        lv = payload + h.rep_len; lv_len = (uint64_t)h.def_len;
        const uint8_t* cv = payload + h.rep_len + h.def_len;
        uint64_t clen = (uint64_t)(h.compressed_size - h.rep_len - h.def_len);
        uint64_t ulen = (uint64_t)(h.uncompressed_size - h.rep_len - h.def_len);
        if (ch->codec == 1 && h.is_compressed) {
          body = (uint8_t*)malloc((size_t)ulen + 1);
          int64_t got = orc_snappy_decompress(cv, clen, body, ulen);
          if (got < 0 || (uint64_t)got != ulen) { rc = fail(ORC_ECORRUPT, "V2 values decompression"); break; }
          vals = body; vals_len = ulen;
        } else {
          if (clen != ulen) { rc = fail(ORC_ECORRUPT, "V2 page sizes differ"); break; }
          vals = cv; vals_len = clen;
        }
      }

      /* definition levels -> validity */
      defs = (uint32_t*)realloc(defs, sizeof(uint32_t) * (size_t)(nv > 0 ? nv : 1));
      int64_t nn = nv;
      if (optional) {
        if (orc_hybrid_decode(lv, lv_len, 1, nv, defs) < 0) { rc = fail(ORC_ECORRUPT, "definition levels truncated"); break; }
        nn = 0;
        for (int64_t i = 0; i < nv; ++i) {
          if (defs[i] > 1) { rc = fail(ORC_ECORRUPT, "definition level above maximum"); break; }
          nn += defs[i];
        }
        if (rc != ORC_OK) break;
        if (h.type == 3 && h.num_nulls != nv - nn) { rc = fail(ORC_ECORRUPT, "V2 null count mismatch"); break; }
      } else {
        for (int64_t i = 0; i < nv; ++i) defs[i] = 1;
        if (h.type == 3 && h.num_nulls != 0) { rc = fail(ORC_ECORRUPT, "nulls in a required column"); break; }
      }

      /* values (non-null only) */
      dvals = (uint64_t*)realloc(dvals, sizeof(uint64_t) * (size_t)(nn > 0 ? nn : 1));
      uint64_t* spos = NULL; uint32_t* slen = NULL; const uint8_t* sbase = NULL;
      int enc = h.encoding;
      if (enc == 0) { /* PLAIN */
        if (type == 6) {
          spos = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nn > 0 ? nn : 1));
          slen = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
          uint64_t q = 0;
          for (int64_t k = 0; k < nn; ++k) {
            if (vals_len - q < 4) { rc = fail(ORC_ECORRUPT, "string length truncated"); break; }
            uint32_t l = (uint32_t)vals[q] | ((uint32_t)vals[q + 1] << 8) | ((uint32_t)vals[q + 2] << 16) | ((uint32_t)vals[q + 3] << 24);
            q += 4;
            if (l > vals_len - q) { rc = fail(ORC_ECORRUPT, "string truncated"); break; }
            spos[k] = q; slen[k] = l;
            q += l;
          }
          sbase = vals;
        } else {
          uint64_t w = (uint64_t)width_of(type);
          if ((uint64_t)nn * w > vals_len) { rc = fail(ORC_ECORRUPT, "PLAIN values truncated"); break; }
          for (int64_t k = 0; k < nn; ++k) {
            uint64_t v = 0;
            for (uint64_t j = 0; j < w; ++j) v |= (uint64_t)vals[(uint64_t)k * w + j] << (8 * j);
            dvals[k] = v;
          }
        }
      } else if (enc == 2 || enc == 8) { /* PLAIN_DICTIONARY / RLE_DICTIONARY */
        if (!have_dict) { rc = fail(ORC_ECORRUPT, "dictionary-encoded page without dictionary"); break; }
        if (nn > 0) {
          if (vals_len < 1) { rc = fail(ORC_ECORRUPT, "missing index bit width"); break; }
          int w = vals[0];
          if (w > 32) { rc = fail(ORC_ECORRUPT, "index bit width above 32"); break; }
          idx = (uint32_t*)realloc(idx, sizeof(uint32_t) * (size_t)nn);
          if (orc_hybrid_decode(vals + 1, vals_len - 1, w, nn, idx) < 0) { rc = fail(ORC_ECORRUPT, "dictionary indices truncated"); break; }
          for (int64_t k = 0; k < nn; ++k) if ((int64_t)idx[k] >= dict.n) { rc = fail(ORC_ECORRUPT, "dictionary index out of range"); break; }
          if (rc != ORC_OK) break;
          if (type == 6) {
            spos = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nn);
            slen = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)nn);
            for (int64_t k = 0; k < nn; ++k) { spos[k] = dict.spos[idx[k]]; slen[k] = dict.slen[idx[k]]; }
            sbase = dict.body;
          } else {
            for (int64_t k = 0; k < nn; ++k) dvals[k] = dict.fixed[idx[k]];
          }
        }
      } else if (enc == 5) { /* DELTA_BINARY_PACKED */
        if (type != 1 && type != 2) { rc = fail(ORC_EUNSUPPORTED, "DELTA_BINARY_PACKED on a non-integer column"); break; }
        if (orc_delta_decode(vals, vals_len, type == 1, nn, dvals) < 0) { rc = fail(ORC_ECORRUPT, "bad DELTA_BINARY_PACKED data"); break; }
      } else if (enc == 6) { /* DELTA_LENGTH_BYTE_ARRAY */
        if (type != 6) { rc = fail(ORC_EUNSUPPORTED, "DELTA_LENGTH_BYTE_ARRAY on a non-string column"); break; }
        spos = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nn > 0 ? nn : 1));
        slen = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
        if (orc_delta_length_decode(vals, vals_len, nn, spos, slen) < 0) { rc = fail(ORC_ECORRUPT, "bad DELTA_LENGTH_BYTE_ARRAY data"); free(spos); free(slen); break; }
        sbase = vals;
      } else if (enc == 7) { /* DELTA_BYTE_ARRAY */
        if (type != 6) { rc = fail(ORC_EUNSUPPORTED, "DELTA_BYTE_ARRAY on a non-string column"); break; }
        spos = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nn > 0 ? nn : 1));
        slen = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
        if (orc_delta_byte_array_decode(vals, vals_len, nn, &mat, &mat_cap, spos, slen) < 0) { rc = fail(ORC_ECORRUPT, "bad DELTA_BYTE_ARRAY data"); free(spos); free(slen); break; }
        sbase = mat;
      } else if (enc == 9) { /* BYTE_STREAM_SPLIT */
        if (type == 6) { rc = fail(ORC_EUNSUPPORTED, "BYTE_STREAM_SPLIT on a string column"); break; }
        if (orc_byte_stream_split_decode(vals, vals_len, width_of(type), nn, dvals) < 0) { rc = fail(ORC_ECORRUPT, "BYTE_STREAM_SPLIT values truncated"); break; }
      } else {
        rc = fail(ORC_EUNSUPPORTED, "unsupported value encoding");
        break;
      }

      /* scatter to rows */
      int64_t k = 0;
      for (int64_t i = 0; i < nv; ++i) {
        int64_t orow = row + i;
        if (type == 6) out->offsets[orow] = out->chars_len;
        if (!defs[i]) continue;
        out->validity[orow >> 3] |= (uint8_t)(1u << (orow & 7));
        if (type == 6) {
          if (!chars_append(out, &chars_cap, sbase + spos[k], slen[k])) { rc = fail(ORC_ENOMEM, "out of memory"); break; }
        } else {
          uint64_t v = dvals[k];
          memcpy((uint8_t*)out->values + (size_t)orow * (size_t)width_of(type), &v, (size_t)width_of(type));
        }
        ++k;
      }
      free(spos); free(slen);
      if (rc != ORC_OK) break;
      row += nv;
      chunk_rows += nv;
      out->pages++;
    }
    if (rc == ORC_OK && chunk_rows != f->rg_rows[g]) rc = fail(ORC_ECORRUPT, "pages do not cover the row group");
  }
  if (type == 6 && out->offsets) out->offsets[rows] = out->chars_len;
  free(defs); free(idx); free(dvals); free(body); free(mat);
  dict_clear(&dict);
  if (rc != ORC_OK) orc_column_free(out);
  return rc;
}
