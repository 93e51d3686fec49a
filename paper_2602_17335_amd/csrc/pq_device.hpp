// pq_device.hpp -- device-side helpers of the GPU scan: bounded byte reads,
// ULEB128/zigzag, Thrift-compact page-header parsing, bit extraction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pq_internal.h"

namespace pqk {

__device__ __forceinline__ void set_err(uint32_t* err, uint32_t code, uint32_t where) {
  atomicCAS(err, 0u, code | (where << 8));
}

// 16-byte cached reader over a 16-byte-aligned base.  Reads round down to a
// 16-byte boundary, so the buffer must be readable up to its length rounded
// up to 16 bytes.
struct BR {
  const uint8_t* base;
  uint64_t cpos;
  uint32_t c0, c1, c2, c3;
  __device__ __forceinline__ void init(const uint8_t* b) {
    base = b;
    cpos = ~0ull;
    c0 = c1 = c2 = c3 = 0;
  }
  __device__ __forceinline__ uint32_t byte(uint64_t off) {
    uint64_t a = off & ~15ull;
    if (a != cpos) {
      uint4 v = *reinterpret_cast<const uint4*>(base + a);
      c0 = v.x; c1 = v.y; c2 = v.z; c3 = v.w;
      cpos = a;
    }
    uint32_t k = (uint32_t)(off & 15);
    uint32_t w = (k < 8) ? ((k < 4) ? c0 : c1) : ((k < 12) ? c2 : c3);
    return (w >> ((k & 3) * 8)) & 0xffu;
  }
  // little-endian u32 at an arbitrary offset
  __device__ __forceinline__ uint32_t u32(uint64_t off) {
    return byte(off) | (byte(off + 1) << 8) | (byte(off + 2) << 16) | (byte(off + 3) << 24);
  }
};

// ULEB128 (at most 10 bytes) from [pos, end), through any reader with byte()
template <class R>
__device__ __forceinline__ uint64_t br_uleb(R& r, uint64_t& pos, uint64_t end, bool& bad) {
  uint64_t v = 0;
  for (int s = 0; s < 70; s += 7) {
    if (pos >= end) { bad = true; return 0; }
    uint32_t b = r.byte(pos++);
    if (s == 63 && (b & 0x7e)) { bad = true; return 0; }
    v |= (uint64_t)(b & 0x7f) << s;
    if (!(b & 0x80)) return v;
  }
  bad = true;
  return 0;
}
__device__ __forceinline__ int64_t unzz(uint64_t v) { return (int64_t)(v >> 1) ^ -(int64_t)(v & 1); }

// Skips one Thrift-compact value of `type` (iterative; nesting depth <= 8).
template <class R>
__device__ inline bool th_skip(R& r, uint64_t& pos, uint64_t end, int type) {
  struct Fr { int is_list; int etype; uint32_t left; };
  Fr st[8];
  int sp = 0;
  bool bad = false;
  int cur = type;
  for (;;) {
    switch (cur) {
      case 1: case 2: break;
      case 3: pos += 1; break;
      case 4: case 5: case 6: br_uleb(r, pos, end, bad); break;
      case 7: pos += 8; break;
      case 8: { uint64_t l = br_uleb(r, pos, end, bad); pos += l; break; }
      case 9: case 10: {
        if (pos >= end) return false;
        uint32_t h = r.byte(pos++);
        uint64_t n = h >> 4;
        if (n == 15) n = br_uleb(r, pos, end, bad);
        if (sp == 8 || n > 0xffffffffull) return false;
        st[sp++] = Fr{1, (int)(h & 15), (uint32_t)n};
        break;
      }
      case 12:
        if (sp == 8) return false;
        st[sp++] = Fr{0, 0, 0};
        break;
      default: return false;
    }
    if (bad || pos > end) return false;
    // next value to consume
    for (;;) {
      if (sp == 0) return true;
      Fr& f = st[sp - 1];
      if (f.is_list) {
        if (f.left == 0) { --sp; continue; }
        f.left--;
        cur = f.etype;
        if (cur == 1 || cur == 2) { pos += 1; if (pos > end) return false; continue; }
        break;
      }
      if (pos >= end) return false;
      uint32_t b = r.byte(pos++);
      if (b == 0) { --sp; continue; }
      cur = b & 15;
      if (!(b >> 4)) br_uleb(r, pos, end, bad);
      if (bad) return false;
      if (cur == 1 || cur == 2) continue;
      break;
    }
  }
}

struct PageHdr {
  int32_t type, unc, comp, nv, enc, nnulls, nrows, def_len, rep_len, is_comp;
  int32_t has_sub;
};

// Parses one Thrift-compact PageHeader starting at pos; pos ends past it
// (through any reader with byte()).
template <class R>
__device__ inline bool parse_page_header(R& r, uint64_t& pos, uint64_t end, PageHdr& h) {
  h.type = -1; h.unc = -1; h.comp = -1; h.nv = -1; h.enc = -1; h.nnulls = 0; h.nrows = -1;
  h.def_len = 0; h.rep_len = 0; h.is_comp = 1; h.has_sub = 0;
  bool bad = false;
  int last = 0;
  for (;;) {
    if (pos >= end) return false;
    uint32_t b = r.byte(pos++);
    if (b == 0) break;
    int t = b & 15, d = b >> 4;
    int id = d ? last + d : (int)unzz(br_uleb(r, pos, end, bad));
    last = id;
    if (bad) return false;
    if (t == 5 && (id == 1 || id == 2 || id == 3)) {
      int32_t v = (int32_t)unzz(br_uleb(r, pos, end, bad));
      if (id == 1) h.type = v; else if (id == 2) h.unc = v; else h.comp = v;
    } else if (t == 12 && (id == 5 || id == 7 || id == 8)) {
      int last2 = 0;
      for (;;) {
        if (pos >= end) return false;
        uint32_t b2 = r.byte(pos++);
        if (b2 == 0) break;
        int t2 = b2 & 15, d2 = b2 >> 4;
        int id2 = d2 ? last2 + d2 : (int)unzz(br_uleb(r, pos, end, bad));
        last2 = id2;
        if (bad) return false;
        if (t2 == 1 || t2 == 2) { if (id == 8 && id2 == 7) h.is_comp = (t2 == 1); continue; }
        if (t2 == 5 && id2 == 1) { h.nv = (int32_t)unzz(br_uleb(r, pos, end, bad)); continue; }
        if (t2 == 5 && id != 8 && id2 == 2) { h.enc = (int32_t)unzz(br_uleb(r, pos, end, bad)); continue; }
        if (t2 == 5 && id == 8 && id2 >= 2 && id2 <= 6) {
          int32_t v = (int32_t)unzz(br_uleb(r, pos, end, bad));
          if (id2 == 2) h.nnulls = v; else if (id2 == 3) h.nrows = v; else if (id2 == 4) h.enc = v;
          else if (id2 == 5) h.def_len = v; else h.rep_len = v;
          continue;
        }
        if (!th_skip(r, pos, end, t2)) return false;
      }
      h.has_sub = 1;
    } else {
      if (!th_skip(r, pos, end, t)) return false;
    }
    if (bad || pos > end) return false;
  }
  return !bad;
}

// Little-endian u32 at any byte offset of a 4-byte-aligned base (two
// aligned loads and a byte funnel shift).
__device__ __forceinline__ uint32_t ld_u32(const uint8_t* base4, uint64_t off) {
  const uint32_t* q = reinterpret_cast<const uint32_t*>(base4 + (off & ~3ull));
  uint32_t s = (uint32_t)(off & 3);
  uint32_t lo = q[0];
  if (!s) return lo;
  return __builtin_amdgcn_alignbyte(q[1], lo, s);
}
__device__ __forceinline__ uint64_t ld_u64(const uint8_t* base4, uint64_t off) {
  const uint32_t* q = reinterpret_cast<const uint32_t*>(base4 + (off & ~3ull));
  uint32_t s = (uint32_t)(off & 3);
  uint32_t a = q[0], b = q[1];
  if (!s) return (uint64_t)a | ((uint64_t)b << 32);
  uint32_t c = q[2];
  return (uint64_t)__builtin_amdgcn_alignbyte(b, a, s) | ((uint64_t)__builtin_amdgcn_alignbyte(c, b, s) << 32);
}

// w bits (w <= 64) starting at absolute bit position `bit` of a 4-byte
// aligned base, least significant bit first.
__device__ __forceinline__ uint64_t get_bits(const uint8_t* base4, uint64_t bit, uint32_t w) {
  if (w == 0) return 0;
  uint64_t dw = bit >> 5;
  uint32_t sh = (uint32_t)(bit & 31);
  const uint32_t* q = reinterpret_cast<const uint32_t*>(base4) + dw;
  uint64_t lo = (uint64_t)q[0] | ((uint64_t)q[1] << 32);
  uint64_t v = lo >> sh;
  if (sh + w > 64) v |= (uint64_t)q[2] << (64 - sh);
  return w == 64 ? v : (v & ((1ull << w) - 1));
}

}  // namespace pqk
