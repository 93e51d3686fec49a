/*
 * pq.h -- C ABI of the MI355X Parquet column-chunk scanner.
 *
 * Scope.  A Parquet file that is already resident in GPU memory is scanned
 * into device-resident columnar buffers: page headers are parsed, Snappy
 * page bodies decompressed, definition levels and dictionary indices decoded
 * from the RLE/bit-packed hybrid, dictionaries gathered, and PLAIN,
 * DELTA_BINARY_PACKED and BYTE_ARRAY values decoded.  This is the GPU scan the
 * paper studies (Sec. 2: row groups -> column chunks -> pages, V1/V2
 * encodings, chunk-level compression, decompression and decoding as GPU
 * kernels; Sec. 3: the page count, row-group size, encoding and compression
 * knobs), applied to files already in HBM.  Supported: flat schemas (no
 * nesting, no REPEATED), physical types INT32, INT64, DOUBLE, BYTE_ARRAY;
 * REQUIRED and OPTIONAL columns; V1 and V2 data pages; PLAIN,
 * PLAIN_DICTIONARY, RLE_DICTIONARY and DELTA_BINARY_PACKED (INT32/INT64;
 * blocks of at most 65536 values in at most 16 miniblocks -- larger blocks
 * are valid Parquet and return PQ_EUNSUPPORTED); BYTE_STREAM_SPLIT (INT32,
 * INT64, DOUBLE); DELTA_LENGTH_BYTE_ARRAY and DELTA_BYTE_ARRAY (strings; a
 * DELTA_BYTE_ARRAY page holding a value longer than 16 KiB returns
 * PQ_EUNSUPPORTED when its column is scanned); codecs UNCOMPRESSED and
 * SNAPPY.
 *
 * Output layout (per selected column, rows of the selected row groups
 * concatenated in row-group order):
 *   values    fixed-width little-endian values, `rows` entries; null rows 0.
 *             DOUBLE is copied as its 64-bit pattern (no floating point).
 *   validity  LSB-first bitmap, bit i of byte i/8, 1 = valid.  The library
 *             writes whole 32-bit words: the buffer must be 4-byte aligned
 *             and hold ((rows+31)/32)*4 bytes; bits past `rows` are 0.
 *             Required for OPTIONAL columns; may be NULL for REQUIRED columns
 *             (a given buffer is then set to all ones).
 *   offsets   BYTE_ARRAY only: rows+1 int64 values, offsets[0] = 0,
 *             offsets[i+1] - offsets[i] = length of row i (0 for nulls).
 *   chars     BYTE_ARRAY only: the concatenated bytes of all valid rows.
 *
 * Pointers.  Every buffer passed to this library is a device pointer unless
 * stated otherwise.  The library never frees caller memory.
 *
 * Errors.  Functions return PQ_OK (0) or a negative pq_status.  Errors the
 * host can detect return before anything is enqueued.  Corruption found by a
 * kernel during a scan sets the error word in that scan's workspace (first
 * error wins); kernels never write outside the caller's buffers, and outputs
 * are undefined after such an error.  pq_scan_check() synchronises the
 * stream and reports it.  pq_last_error() gives a thread-local message for
 * the last failure.
 *
 * Concurrency.  One handle may be scanned concurrently on several streams,
 * each scan with its own workspace (and so its own error word).  The handle
 * is read-only after pq_open_device returns.
 */
#ifndef PQ_H
#define PQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pq_file_s* pq_file;
typedef void* pq_stream; /* a hipStream_t; NULL = the null stream */

typedef enum {
  PQ_OK = 0,
  PQ_EINVAL = -1,       /* bad argument (NULL pointer, range, mask) */
  PQ_ECORRUPT = -2,     /* the file violates the format */
  PQ_EUNSUPPORTED = -3, /* valid Parquet outside the supported subset */
  PQ_ENOMEM = -4,       /* device or host allocation failed */
  PQ_EHIP = -5,         /* a HIP runtime call failed */
  PQ_ECAPACITY = -7,    /* an output or workspace buffer is smaller than planned */
  PQ_EBUSY = -8         /* the server has not finished the request within the wait */
} pq_status;

typedef enum { PQ_INT32 = 1, PQ_INT64 = 2, PQ_DOUBLE = 5, PQ_BYTE_ARRAY = 6 } pq_type;

typedef struct {
  int32_t type;     /* pq_type */
  int32_t nullable; /* 1 = OPTIONAL, 0 = REQUIRED */
  char name[64];    /* leaf name, truncated to 63 bytes */
} pq_column_info;

/* Sizes of one scan, filled by pq_plan(). */
typedef struct {
  int64_t rows;               /* output rows: sum of the selected row groups */
  uint64_t workspace_bytes;   /* device workspace pq_plan/pq_scan need */
  int64_t chars_bytes[64];    /* per selected column (in mask order); -1 until known */
} pq_scan_sizes;

/* Output buffers of one selected column. */
typedef struct {
  void* values;          /* fixed-width columns: rows * width bytes */
  uint8_t* validity;     /* ((rows+31)/32)*4 bytes, 4-byte aligned; NULL only for REQUIRED */
  int64_t* offsets;      /* BYTE_ARRAY: rows+1 */
  uint8_t* chars;        /* BYTE_ARRAY */
  uint64_t chars_capacity;
} pq_column_out;

/* Statistics of an opened file (page table, tile index and resident
   dictionaries built at open). */
typedef struct {
  int64_t pages;          /* data pages */
  int64_t dict_pages;
  int64_t tiles;          /* decode tiles (row ranges of one page) */
  int64_t compressed_pages;
  uint64_t encoded_bytes; /* sum of compressed page payload sizes */
  uint64_t uncompressed_bytes;
  double open_ms_device;  /* time of the open-time passes: page walk and tile
                             index (device events), dictionaries and tile
                             prefix (host clock) */
  uint64_t device_bytes;  /* device memory the handle holds until pq_close
                             (index, checkpoints, resident dictionaries) */
} pq_file_stats;

/*
 * Opens a Parquet file that lies in device memory (Sec. 2: the file is read
 * as row groups of column chunks, each chunk a sequence of pages).
 *   dev_buf  device pointer to the whole file (borrowed: it must stay valid
 *            and unmodified until pq_close; it is never written).  It must be
 *            readable up to `len` rounded up to a multiple of 16 bytes, which
 *            every HIP and PyTorch allocation is.
 *   len      file length in bytes.
 *   stream   stream used for the open-time kernels; the call synchronises it
 *            (a caller that owns its streams keeps the open off the default
 *            stream).
 *   out      receives the handle.
 * The footer is copied to the host and decoded there (file layout and
 * Thrift-compact metadata, Sec. 2's row-group/chunk/page hierarchy); kernels
 * then walk every column chunk's page headers into a device page table and
 * build the tile index (entry positions of every fixed-size row tile in the
 * level and value streams of each page, with checkpoints inside the tile)
 * that lets a scan start decoding at any tile.  The index is built in
 * passes: the dictionary pages first, then runs of data pages whose
 * decompressed bytes fit a 512 MiB window, each pass's compressed pages
 * decompressed into that window.  Every dictionary page is decoded once into
 * a resident dictionary kept by the handle (fixed-width arrays; string
 * positions, lengths and 64-byte slots), so scans never rebuild one.  Last,
 * the tile prefix: for every column with DELTA_BINARY_PACKED or BYTE_ARRAY
 * pages, a pass over its tiles (after decompression and dictionary decode,
 * in batches of row groups, or of pages, with at most 512 MiB of temporary
 * device memory) counts each tile's DELTA sum or string bytes, and their
 * exclusive prefix sum over the file's tiles is kept on the device and the
 * host (8 bytes per tile).  A scan takes DELTA carries and string offsets from
 * it, and pq_plan the chars sizes.  Returns PQ_ECORRUPT for a malformed file
 * (including corrupt level, DELTA, dictionary-index or string data found by
 * the index or prefix passes), PQ_EUNSUPPORTED for valid files outside the
 * supported subset.
 */
pq_status pq_open_device(const void* dev_buf, uint64_t len, pq_stream stream, pq_file* out);

/* Metadata of an opened file (Sec. 2: row groups, one column chunk per
   column and row group).  Host-only; PQ_EINVAL for a NULL argument or an
   index out of range. */
pq_status pq_num_row_groups(pq_file f, int32_t* n);
pq_status pq_num_columns(pq_file f, int32_t* n);
pq_status pq_column_info_get(pq_file f, int32_t col, pq_column_info* out);
pq_status pq_row_group_rows(pq_file f, int32_t rg, int64_t* rows);
/* Sizes and open time of the file's page table and index (Sec. 3: the page
   count and row-group size knobs show up as pages and tiles). */
pq_status pq_file_stats_get(pq_file f, pq_file_stats* out);

/*
 * Sizes a scan (Sec. 2: a scan reads the selected column chunks of a range
 * of row groups) of columns `col_mask` (bit i = leaf column i, at most 64
 * columns) over row groups [rg_begin, rg_end): rows, workspace_bytes, and
 * chars_bytes (exact chars bytes of each BYTE_ARRAY column, 0 for the
 * others).  Host-only: the string byte counts come from the tile prefix
 * that pq_open_device builds, so no GPU work is enqueued and nothing is
 * synchronised.  PQ_EINVAL for a bad range or mask.
 */
pq_status pq_plan(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end, pq_scan_sizes* out);

/*
 * Enqueues the scan on `stream` and returns without synchronising (Sec. 2:
 * decompression, then decoding, both as GPU kernels).
 *   outs       host array of n_outs descriptors; outs[k] belongs to the k-th
 *              set bit of col_mask in ascending order.
 *   workspace  device buffer of at least the planned workspace_bytes, owned
 *              by the caller, not used by anything else until the scan ends.
 * Steps enqueued: the workspace header (cleared error word, column table) in
 * one host-to-device copy; Snappy decompression of compressed data pages
 * into the workspace; offsets[rows] and the chars capacity check of string
 * columns (from the tile prefix built at open); then the decode kernels
 * (definition levels -> validity and ranks, dictionary indices -> gather,
 * PLAIN, DELTA_BINARY_PACKED with carries from the tile prefix, BYTE_ARRAY ->
 * offsets and chars).  A chars buffer smaller than the decoded strings
 * is reported by pq_scan_check() as PQ_ECAPACITY (no chars
 * are written for the tiles that would overflow; nothing is written past
 * chars_capacity).
 */
pq_status pq_scan(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end, const pq_column_out* outs,
                  int32_t n_outs, void* workspace, uint64_t workspace_bytes, pq_stream stream);
/* The workspace must be 256-byte aligned.  values must be aligned to the
   value width.  Returns PQ_EINVAL / PQ_ECAPACITY (workspace) before
   enqueueing anything. */

/*
 * pq_scan without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same scan as pq_scan, with the workspace taken
 * from a file-scope device array of 64 MiB that every GPU the library runs
 * on holds until the process ends; its device address is looked up once per
 * device (hipGetSymbolAddress) on the first call made with that device
 * current.  The caller still passes the outputs.  Calls no hipMalloc,
 * hipFree or other device-memory allocator.  Returns PQ_ECAPACITY, before
 * enqueueing anything, when the scan's planned workspace (pq_plan) exceeds
 * 64 MiB -- a scan of compressed pages needs their decompressed bytes there.
 * Every call on one GPU shares that GPU's array (the last call's contents
 * stay; the scan's header, with its cleared error word, is rewritten by
 * each call): calls that overlap on one GPU race, so a caller serialises
 * them (one stream, or its own ordering).  pq_scan_check(f, NULL, stream)
 * reports the error word of the last such scan on the current device.
 */
pq_status pq_scan_noalloc(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end, const pq_column_out* outs,
                          int32_t n_outs, pq_stream stream);

/*
 * A file held in host memory, scanned with its row groups streamed to the
 * device (Sec. 4.1: an overlapped reader decodes row group by row group
 * while the next row group is transferred, instead of waiting for the whole
 * file).  pq_open_host copies the file to a temporary device buffer for the
 * open-time passes (page table, tile index, dictionaries -- all copied into
 * the handle -- and tile prefix) and frees it; host_buf is borrowed until
 * pq_close and should be pinned (hipHostMalloc, or a pinned torch tensor),
 * or the copies cannot overlap.  pq_plan of such a handle includes in
 * workspace_bytes two staging slots (each the largest row group's selected
 * chunks) and a column table per row group.  pq_scan, pq_scan_noalloc and
 * the batch calls refuse such a handle (PQ_EINVAL).
 */
pq_status pq_open_host(const void* host_buf, uint64_t len, pq_stream stream, pq_file* out);

/* The scan of a host-resident file (Sec. 4.1, overlapped reading): the
   selected column chunks of each row group are copied into a staging slot
   of the workspace on `copy_stream`, while `stream` decompresses and
   decodes the previous row group from the other slot; events order each
   slot's reuse.  Outputs, errors and pq_scan_check as for pq_scan.  With
   the two streams equal nothing overlaps (still correct); every copy is waited on by `stream`, so the scan
   is complete once `stream` is.  Calls on one handle are issued from one
   host thread at a time (the handle keeps the slot events). */
pq_status pq_scan_streamed(pq_file f, uint64_t col_mask, int32_t rg_begin, int32_t rg_end, const pq_column_out* outs,
                           int32_t n_outs, void* workspace, uint64_t workspace_bytes, pq_stream copy_stream,
                           pq_stream stream);

/* Synchronises `stream` and returns (then clears) the error word of the
   scan that last used `workspace` (Sec. 2: the decode kernels of that
   scan): PQ_OK, or PQ_ECORRUPT / PQ_EUNSUPPORTED / PQ_ECAPACITY found by a
   kernel.  Scans on other workspaces are not affected.  `f` may be NULL
   (a batch over several files); `workspace` NULL means the scratch array of
   pq_scan_noalloc on the current device. */
pq_status pq_scan_check(pq_file f, const void* workspace, pq_stream stream);

/* Encoded bytes of column `col` over all row groups (Sec. 3: the encoded
   size that the encoding and compression knobs change): data-page payloads
   (levels + values as stored) and dictionary-page payloads. */
pq_status pq_column_bytes(pq_file f, int32_t col, uint64_t* data_bytes, uint64_t* dict_bytes);

/* Encodings used by the data pages of column `col` over all row groups
   (Sec. 2: V1 and V2 encodings may differ page by page)
   (the page header's encoding field, Parquet's Encoding enum: PLAIN 0,
   PLAIN_DICTIONARY 2, DELTA_BINARY_PACKED 5, RLE_DICTIONARY 8): bit e of
   *mask is set when some data page uses encoding e.  Host-only. */
pq_status pq_column_encodings(pq_file f, int32_t col, uint32_t* mask);

/* Measurement hook (Sec. 3: the effective bandwidth of a scan is the decoded
   bytes over its run time).  While enabled, every kernel pq_scan enqueues on a
   handle (f NULL: every kernel of a batched scan) is bracketed by a pair of
   HIP events on the scan's stream;
   pq_profile_read() waits for the recorded events and returns, per kernel
   name, the number of launches and the summed device time since the last
   pq_profile(f, 1).  pq_profile(f, 0) stops recording. */
typedef struct {
  char name[32];
  uint64_t launches;
  double total_ms;
} pq_kernel_time;
pq_status pq_profile(pq_file f, int32_t enable);
pq_status pq_profile_read(pq_file f, pq_kernel_time* out, int32_t capacity, int32_t* n);

/* Measurement reference (Sec. 3's effective bandwidth is compared with what
   the memory system sustains): enqueues a plain streaming copy of `bytes`
   bytes from device buffer src to device buffer dst on `stream` (16-byte
   loads, non-temporal 16-byte stores; the buffers must not overlap and
   should be 16-byte aligned).  The copy's bytes over its time are the
   practical ceiling a scan's encoded-plus-decoded bytes are reported
   against ("% of copy"). */
pq_status pq_copy_probe(void* dst, const void* src, uint64_t bytes, pq_stream stream);

/*
 * Batched scans: several requests, over one or several opened files, in one
 * set of launches (Sec. 3, Insight 1: a GPU decoder needs many independent
 * pages in one launch to fill the chip; files with small row groups offer
 * few pages each).
 *
 * One request: columns `col_mask` of row groups [rg_begin, rg_end) of
 * `file`, into `outs` (one descriptor per set bit, ascending, as for
 * pq_scan; may be NULL for pq_plan_batch).
 */
typedef struct {
  pq_file file;
  uint64_t col_mask;
  int32_t rg_begin, rg_end;
  const pq_column_out* outs;
} pq_request;

/* Work classes of the schedule: decoder kind (9: PLAIN / dictionary /
   BYTE_STREAM_SPLIT 4- and 8-byte values, DELTA_BINARY_PACKED, strings,
   strings of slot dictionaries) x dictionary-index width (2: up to 12 bits,
   wider) x page size (3: one tile, 2-16 tiles, more). */
#define PQ_TUNE_CLASSES 54
#define PQ_FORM_BATCHED 0  /* one persistent decode launch over a work queue */
#define PQ_FORM_PER_PAGE 1 /* one launch per page and decoder (the plain form) */
typedef struct {
  int32_t form;          /* PQ_FORM_BATCHED or PQ_FORM_PER_PAGE */
  int32_t waves_per_cu;  /* persistent grid: waves per compute unit, 1..16 (0: 8) */
  int32_t queues;        /* 8: one work queue per XCD, column chunks spread over them by
                            cost (longest first); 1: one shared queue in request order
                            (0: 8) */
  int32_t pad_;
  uint8_t tiles_per_unit[PQ_TUNE_CLASSES]; /* tiles a wave takes per queue grab, per
                                              class, 1..64 (0: 2) */
  uint8_t pad2_[2];
} pq_tuning;

/* The default schedule (every field at its default). */
pq_status pq_tuning_default(pq_tuning* out);

/* Sizes a batch (Sec. 2: each request reads the selected column chunks of
   its row groups): the workspace bytes and, for every selected column of
   every request in order (request 0's columns ascending, then request 1's,
   ...), its exact chars bytes (0 for fixed-width columns) in chars_bytes
   (capacity n_chars entries; PQ_EINVAL if it is smaller).  Host-only. */
pq_status pq_plan_batch(const pq_request* reqs, int32_t n, uint64_t* workspace_bytes, int64_t* chars_bytes,
                        int32_t n_chars);

/* Enqueues a batch on `stream` (Sec. 2: decompression, then decoding, as GPU
   kernels; Sec. 3, Insight 1: the pages of every request form one grid of
   work).  With PQ_FORM_BATCHED: Snappy decompression of every compressed
   data page (one launch for the page-sequential decoder, one for the
   block-parallel one), the string totals, one persistent decode launch
   whose waves take work units from the queues, and the shared validity
   words of OPTIONAL columns.  With PQ_FORM_PER_PAGE the same work is one
   launch per page instead.  `tuning` NULL = the default schedule.  Errors
   as for pq_scan; pq_scan_check(NULL, workspace, stream) reports device
   errors.  Requests must not write overlapping outputs. */
pq_status pq_scan_batch(const pq_request* reqs, int32_t n, const pq_tuning* tuning, void* workspace,
                        uint64_t workspace_bytes, pq_stream stream);

/* Autotuner of the batched form's schedule (Sec. 3, Insight 1: the page to
   grid mapping decides how well a decode launch fills the GPU).  Runs the
   batch with candidate schedules on `stream` -- coordinate descent over the
   queue layout, the waves per CU, and the tiles per unit of every work class
   present, largest classes first -- timing each candidate as the median of
   `reps` runs between HIP events, and returns the fastest in *best with its
   time (and the default schedule's) in milliseconds.  Synchronises the
   stream; the outputs hold the batch's result afterwards. */
pq_status pq_autotune_batch(const pq_request* reqs, int32_t n, void* workspace, uint64_t workspace_bytes,
                            pq_stream stream, int32_t reps, pq_tuning* best, double* best_ms, double* default_ms);

/*
 * The scan server: a request loop over a catalog of opened (resident) files
 * for many concurrent clients (Sec. 4: overlapping the reader's stages with
 * other GPU work; Sec. 4.2: consumers take row groups as they are
 * produced).  Requests -- columns of a row-group range of one catalog file
 * -- are admitted in arrival order against a device-memory budget: each
 * needs its outputs and its share of a batch workspace in the server's one
 * arena of budget_bytes.  A scheduler thread keeps up to `slots` batched
 * scans (pq_scan_batch, at most max_batch requests each, `tuning` NULL = the
 * default schedule) in flight, one per stream: requests that arrive while
 * batches run are batched as soon as a slot and memory are free, so their
 * work overlaps on the device (continuous batching).  Results stay resident
 * in the arena until released; a request identical to a resident (or
 * in-flight) one shares its result.  Unreferenced resident results are
 * evicted, least recently used first, when memory is needed.  Dictionaries
 * are those the handles keep resident.
 */
typedef struct pq_server_s* pq_server;
typedef struct {
  int32_t status;          /* PQ_OK or the request's error */
  int32_t n_outs;          /* selected columns */
  int32_t shared;          /* 1: served by a resident (or in-flight) identical result */
  int32_t pad_;
  int64_t rows;
  uint64_t decoded_bytes;  /* values (null slots included), validity, offsets, chars */
  double queue_ms;         /* submit -> admitted into a batch */
  double latency_ms;       /* submit -> the batch that decoded it finished on the device */
  pq_column_out outs[64];  /* device pointers into the server's arena (layout as pq_scan's),
                              valid until pq_server_release */
} pq_served;
typedef struct {
  uint64_t submitted, completed, failed, batches, cache_hits, evictions;
  uint64_t decoded_bytes;  /* of completed requests */
  uint64_t budget_bytes, used_bytes, resident_results;
} pq_server_stats;

/* Creates a server over n_files opened files (borrowed: they must outlive
   the server), allocating its arena of budget_bytes and `slots` streams
   (1..16). */
pq_status pq_server_create(const pq_file* files, int32_t n_files, uint64_t budget_bytes, int32_t slots,
                           int32_t max_batch, const pq_tuning* tuning, pq_server* out);
/* Queues a request (Sec. 2: columns of a row-group range); thread-safe.
   PQ_EINVAL for a bad file index, range or mask. */
pq_status pq_server_submit(pq_server s, int32_t file, uint64_t col_mask, int32_t rg_begin, int32_t rg_end,
                           uint64_t* id);
/* Waits up to timeout_ms (negative: an hour) for request `id` (Sec. 3: the
   scan's run time is what the effective bandwidth divides by) and fills
   *out; returns the request's status, or PQ_EBUSY on time-out. */
pq_status pq_server_wait(pq_server s, uint64_t id, int32_t timeout_ms, pq_served* out);
/* Releases a finished request's hold on its result, which stays resident
   until evicted (Sec. 4: results stay in GPU memory for the operators that
   consume them). */
pq_status pq_server_release(pq_server s, uint64_t id);
/* Counters of the server (Sec. 3: decoded bytes over time). */
pq_status pq_server_stats_get(pq_server s, pq_server_stats* out);
/* Drains the requests in flight, then frees the arena and the streams
   (Sec. 2: the reader's state). */
void pq_server_destroy(pq_server s);
/* Thread-local message of the server's last failure (Sec. 2: the reader's
   error reporting). */
const char* pq_server_last_error(void);

/* Frees the handle's host and device memory (not dev_buf).  Sec. 2: the
   handle is the reader's state for one file. */
void pq_close(pq_file f);

/* Thread-local description of the last error (Sec. 2: the reader's error
   reporting; no paper passage constrains it further). */
const char* pq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PQ_H */
