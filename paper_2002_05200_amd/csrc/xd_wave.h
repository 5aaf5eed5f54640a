// xd_wave.h -- wavefront-level value types for gfx950 (CDNA4, wave64).
//
// The extension kernel is written at wavefront level: a `vint` is one 32-bit
// value per lane (a VGPR), a `vbool` is one predicate per lane (an EXEC-style
// lane mask), and plain integers are wave-uniform (SGPRs).  Every function
// here is a thin, force-inlined wrapper over a plain expression or a gfx950
// builtin, so the kernel compiles to straight VALU/SALU code:
//   from_prev_lane / from_next_lane  -> v_mov_b32_dpp wave_shr:1 / wave_shl:1
//   ballot / lanes                   -> v_cmp into an SGPR pair / that pair as VCC
//   readlane                         -> v_readlane_b32
//   from_lane                        -> ds_bpermute_b32
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define XD_FN __device__ __forceinline__
#define XD_HD __host__ __device__
#define XD_MEMBER __device__ __forceinline__

namespace xd {

constexpr int kWave = 64;

struct vint { int32_t x; };
// A lane predicate is a plain bool: as a one-member struct it would be
// passed through memory (i1 stored, i8 loaded) and end up in LDS.
using vbool = bool;

XD_FN vint splat(int32_t s) { return {s}; }
XD_FN vint lane_index() { return {(int32_t)__lane_id()}; }
XD_FN int lane_id() { return (int)__lane_id(); }

XD_FN vint operator+(vint a, vint b) { return {a.x + b.x}; }
XD_FN vint operator+(vint a, int32_t b) { return {a.x + b}; }
XD_FN vint operator-(vint a, vint b) { return {a.x - b.x}; }
XD_FN vint operator-(vint a, int32_t b) { return {a.x - b}; }
XD_FN vint operator*(vint a, int32_t b) { return {a.x * b}; }
XD_FN vint operator&(vint a, int32_t b) { return {a.x & b}; }
XD_FN vint operator|(vint a, vint b) { return {a.x | b.x}; }
XD_FN vint operator^(vint a, vint b) { return {a.x ^ b.x}; }
XD_FN vint operator<<(vint a, int s) { return {(int32_t)((uint32_t)a.x << s)}; }
XD_FN vint shr_u(vint a, int s) { return {(int32_t)((uint32_t)a.x >> s)}; }
XD_FN vint shr_s(vint a, int s) { return {a.x >> s}; }
XD_FN vint not_(vint a) { return {~a.x}; }

XD_FN vbool operator>=(vint a, int32_t s) { return a.x >= s; }
XD_FN vbool operator>(vint a, int32_t s) { return a.x > s; }
XD_FN vbool operator==(vint a, int32_t s) { return a.x == s; }
XD_FN vbool operator!=(vint a, int32_t s) { return a.x != s; }
XD_FN vbool both(vbool a, vbool b) { return a & b; }
XD_FN vbool le_u(vint a, uint32_t s) { return (uint32_t)a.x <= s; }

// a[23:0] * b + c (v_mad_u32_u24)
XD_FN vint mad24(vint a, int32_t b, vint c) {
  return {(int32_t)((uint32_t)(a.x & 0xffffff) * (uint32_t)(b & 0xffffff) + (uint32_t)c.x)};
}
XD_FN vint vmax(vint a, vint b) { return {a.x > b.x ? a.x : b.x}; }
XD_FN vint vmax3(vint a, vint b, vint c) { return vmax(vmax(a, b), c); }
XD_FN vint vmin(vint a, vint b) { return {a.x < b.x ? a.x : b.x}; }
XD_FN vint clamp(vint a, int32_t lo, int32_t hi) { return {a.x < lo ? lo : (a.x > hi ? hi : a.x)}; }
XD_FN vint select(vbool p, vint a, vint b) { return {p ? a.x : b.x}; }
XD_FN vint select(vbool p, vint a, int32_t b) { return {p ? a.x : b}; }
XD_FN vint bit_if(vbool p, int bit) { return {p ? (1 << bit) : 0}; }

// unsigned bit-field extract of `width` bits at `pos` (v_bfe_u32)
XD_FN vint bfe_u(vint w, int pos, int width) {
  return {(int32_t)__builtin_amdgcn_ubfe((uint32_t)w.x, (uint32_t)pos, (uint32_t)width)};
}
// signed bit-field extract (v_bfe_i32)
XD_FN vint bfe_s(vint w, int pos, int width) {
  return {(int32_t)__builtin_amdgcn_sbfe(w.x, (uint32_t)pos, (uint32_t)width)};
}
// low 32 bits of ({hi, lo} >> shift), shift in [0, 31] (v_alignbit_b32)
XD_FN vint funnel_shr(vint hi, vint lo, vint shift) {
  return {(int32_t)__builtin_amdgcn_alignbit((uint32_t)hi.x, (uint32_t)lo.x, (uint32_t)shift.x)};
}
XD_FN vint bit_reverse(vint a) { return {(int32_t)__builtin_bitreverse32((uint32_t)a.x)}; }
// (m & a) | (~m & b)  (v_bfi_b32)
XD_FN vint bit_insert(vint m, int32_t a, int32_t b) {
  return {(int32_t)(((uint32_t)m.x & (uint32_t)a) | (~(uint32_t)m.x & (uint32_t)b))};
}

XD_FN uint64_t ballot(vbool p) { return __builtin_amdgcn_ballot_w64(p); }
XD_FN vbool lanes(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }
XD_FN int32_t readlane(vint a, int lane) { return __builtin_amdgcn_readlane(a.x, lane); }
XD_FN int32_t uniform(int32_t s) { return __builtin_amdgcn_readfirstlane(s); }

// lane t receives lane t-1's value; lane 0 receives `fill`
XD_FN vint from_prev_lane(vint a, int32_t fill) {
  return {__builtin_amdgcn_update_dpp(fill, a.x, 0x138, 0xf, 0xf, false)};
}
// lane t receives lane t+1's value; lane 63 receives `fill`
XD_FN vint from_next_lane(vint a, int32_t fill) {
  return {__builtin_amdgcn_update_dpp(fill, a.x, 0x130, 0xf, 0xf, false)};
}
// whole-wave rotations: lane t receives lane t-1 (lane 0 receives lane 63),
// resp. lane t+1 (lane 63 receives lane 0)  -> wave_ror:1 / wave_rol:1
// (every lane is written, so no "old" value is needed)
XD_FN vint rot_prev(vint a) { return {__builtin_amdgcn_mov_dpp(a.x, 0x13c, 0xf, 0xf, false)}; }
XD_FN vint rot_next(vint a) { return {__builtin_amdgcn_mov_dpp(a.x, 0x134, 0xf, 0xf, false)}; }
// lane t receives lane (t + delta)'s value, `fill` where that lane does not exist
XD_FN vint from_lane_offset(vint a, int delta, int32_t fill) {
  int src = lane_id() + delta;
  int got = __builtin_amdgcn_ds_bpermute(src << 2, a.x);
  return {(src >= 0 && src < kWave) ? got : fill};
}

// Per-lane load of words[idx] (idx is clamped by the caller).
XD_FN vint load_word(const uint32_t *words, vint idx) {
  return {(int32_t)words[idx.x]};
}

// Per-job save memory: a store by the first lane only, one int32 per lane
// stored or loaded at per-lane indices, and an atomic add by the first lane
// whose old value every lane receives.
XD_FN void store_first(int32_t *p, int32_t v) {
  if (__lane_id() == 0) *p = v;
}
XD_FN void store_vec(int32_t *base, vint idx, vint v) { base[idx.x] = v.x; }
XD_FN vint load_vec(const int32_t *base, vint idx) { return {base[idx.x]}; }
XD_FN uint32_t atomic_add_first(unsigned long long *p, unsigned long long v) {
  uint32_t old = 0;
  if (__lane_id() == 0) old = (uint32_t)atomicAdd(p, v);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)old);
}

XD_FN int ctz64(uint64_t m) { return __builtin_ctzll(m); }
XD_FN int last_bit64(uint64_t m) { return 63 - __builtin_clzll(m); }
XD_FN int ctz32(uint32_t m) { return __builtin_ctz(m); }
XD_FN int last_bit32(uint32_t m) { return 31 - __builtin_clz(m); }
XD_FN uint64_t lane_range_mask(int lo, int hi) {  // bits lo..hi, 0 <= lo <= hi <= 63
  int w = hi - lo + 1;
  uint64_t m = (w >= 64) ? ~0ull : ((1ull << w) - 1ull);
  return m << lo;
}

}  // namespace xd
