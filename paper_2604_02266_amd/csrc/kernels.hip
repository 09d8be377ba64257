// HIP kernels for gfx950: the structured-sparse DD channel (paper Sec. IV-B) and
// conjugate-gradient LMMSE equalisation (Sec. IV-C, Algorithm 1).
//
// Operator.  For path p with signed bin shifts (tau_p, nu_p), output bin (k, l) of y = H x
// gathers the source bin (<k - tau_p>_M, <l - nu_p>_N) -- the column map r_p(q) of
// Eq. map_chMatDD_col -- with coefficient D_{p,q} = h_p gamma_{p,q} (Eq. D_definition):
//     D = R_p[k] * W[l0]^n,  R_p[k] = h_p e^{j 2 pi nu_p (k - tau_p) / (MN)},
//     W[l0] = e^{j 2 pi l0 / N},  n = floor((k - tau_p) / M) in {-1, 0, 1},
// where l0 is the Doppler bin of the source (the column), n the delay wrap count and the
// product is the twisted phase of Sec. IV-B.  H^H (Eq. sparse_herm_mvm) gathers at the
// inverse map q_p(r) = (<k + tau_p>_M, <l + nu_p>_N) of Eq. herm_mapping with the
// conjugate coefficient of the gathered row.  Both are gather-multiply-reduce over paths:
// no atomics, no dense matrix.
//
// Thread layout.  A workgroup owns a band of Doppler rows of one frame.  Each thread keeps
// one delay column k fixed while it walks the rows of the band, so the P coefficients
// R_p[k], the source columns and the wrap counts of that column are loaded once and stay
// in registers; for a fixed (row, path) the 64 lanes of a wave read 64 consecutive delay
// bins of one source row (one wrap point at most): coalesced complex64 loads.  No MFMA:
// the operator is a sparse gather, not a dense contraction.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "otfs_internal.h"

namespace otfs {
namespace {

// ---------------------------------------------------------------------------------------
// small complex helpers
// ---------------------------------------------------------------------------------------
// explicit fused multiply-adds: the rounding does not depend on how the compiler would
// contract the expression in each kernel, so every kernel forms the same coefficients
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ void cmacf(float2& acc, float2 c, float2 v) {
  acc.x = fmaf(c.x, v.x, acc.x);
  acc.x = fmaf(-c.y, v.y, acc.x);
  acc.y = fmaf(c.x, v.y, acc.y);
  acc.y = fmaf(c.y, v.x, acc.y);
}
__device__ __forceinline__ double2 cmuld(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ void cmacd(double2& acc, double2 c, double2 v) {
  acc.x = fma(c.x, v.x, acc.x);
  acc.x = fma(-c.y, v.y, acc.x);
  acc.y = fma(c.x, v.y, acc.y);
  acc.y = fma(c.y, v.x, acc.y);
}
// bf16 pair (re in the low half, im in the high half) -> complex64
__device__ __forceinline__ float2 bf16x2_to_f2(uint32_t w) {
  return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}
// round-to-nearest-even float -> bf16 bits
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float2 load_y(const void* y, int64_t i, bool bf16) {
  if (bf16) return bf16x2_to_f2(static_cast<const uint32_t*>(y)[i]);
  return static_cast<const float2*>(y)[i];
}
// c + s * p, one rounding per component (used identically wherever a value is recomputed)
__device__ __forceinline__ float2 axpyf(float s, float2 p, float2 c) {
  return make_float2(fmaf(s, p.x, c.x), fmaf(s, p.y, c.y));
}

// ---------------------------------------------------------------------------------------
// memory views
// ---------------------------------------------------------------------------------------
// Pointers kept in frame descriptors are generic; these casts tell the compiler which
// memory they address, so that accesses become global (not flat) instructions, and
// wave-uniform table reads through a constant view become scalar loads.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
using kptr = __attribute__((address_space(4))) T*;
template <class T>
using lptr = __attribute__((address_space(3))) T*;
template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}
typedef unsigned long long u64;
// 8-byte pairs (complex64, int pairs) are moved as 64-bit words through these views.
struct GPairs {   // global table
  gptr<const u64> p;
  __device__ __forceinline__ float2 f(int64_t i) const { return __builtin_bit_cast(float2, p[i]); }
};
struct KPairs {   // wave-uniform table: scalar loads
  kptr<const u64> p;
  __device__ __forceinline__ float2 f(int i) const { return __builtin_bit_cast(float2, p[i]); }
  __device__ __forceinline__ int2 i2(int i) const { return __builtin_bit_cast(int2, p[i]); }
};
struct LdsC {     // complex64 array in LDS
  lptr<u64> p;
  __device__ __forceinline__ float2 ld(int i) const { return __builtin_bit_cast(float2, p[i]); }
  __device__ __forceinline__ void st(int i, float2 v) const { p[i] = __builtin_bit_cast(u64, v); }
  __device__ __forceinline__ LdsC operator+(int o) const { return LdsC{p + o}; }
};
__device__ __forceinline__ GPairs gpairs(const void* t) { return GPairs{(gptr<const u64>)t}; }
__device__ __forceinline__ KPairs kpairs(const void* t) { return KPairs{(kptr<const u64>)t}; }
__device__ __forceinline__ LdsC lds_c(void* t) { return LdsC{(lptr<u64>)t}; }

// A vector of `bytes` bytes read through a buffer resource: the base stays in SGPRs and
// each read takes one 32-bit byte offset (frames hold at most 2^28 elements, so every
// offset fits).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, int64_t bytes) {
  const uint32_t n = bytes > 0xffffffffLL ? 0xffffffffu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, 0x00020000);
}

// Source views of a band application: load(i) issues the reads of element i, value(raw)
// forms the element from them; load_b(vb, sb) reads the element at byte offset vb + sb of
// a complex64 vector, where sb is the same for the whole wave when the caller can prove
// it (it then goes into the instruction's scalar offset).  A stageable view also names the kNV complex64 vectors it
// reads (rsrc(j)) and forms the element from their values (combine); own(i, v) reads them
// at element i.
__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, uint32_t i) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, 0));
}
__device__ __forceinline__ float2 buf_ld2b(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vb, sb, 0));
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// Two adjacent complex64 elements moved as one 16-byte access (the paired gathers).
template <int POLICY = 0>
__device__ __forceinline__ u32x4 buf_ld4b(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
  return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, vb, sb, POLICY));
}
__device__ __forceinline__ void unpack2(u32x4 v, float2& a, float2& b) {
  a = __builtin_bit_cast(float2, u32x2{v.x, v.y});
  b = __builtin_bit_cast(float2, u32x2{v.z, v.w});
}
__device__ __forceinline__ u32x4 pack2(float2 a, float2 b) {
  const u32x2 x = __builtin_bit_cast(u32x2, a), y = __builtin_bit_cast(u32x2, b);
  return u32x4{x.x, x.y, y.x, y.y};
}
struct SrcBuf {   // complex64 vector
  __amdgpu_buffer_rsrc_t r;
  static constexpr int kNV = 1;
  static constexpr bool kStageable = true;
  static constexpr bool kPairs = true;
  using Raw = float2;
  using Raw2 = u32x4;
  __device__ __forceinline__ Raw load(uint32_t i) const { return buf_ld2(r, i); }
  __device__ __forceinline__ Raw load_b(uint32_t vb, uint32_t sb) const { return buf_ld2b(r, vb, sb); }
  __device__ __forceinline__ float2 value(Raw v) const { return v; }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int) const { return r; }
  __device__ __forceinline__ float2 combine(const float2* v) const { return v[0]; }
  __device__ __forceinline__ void own(uint32_t i, float2* v) const { v[0] = buf_ld2(r, i); }
  // pairs: the elements at byte offsets vb + sb and vb + sb + 8
  __device__ __forceinline__ Raw2 load2_b(uint32_t vb, uint32_t sb) const { return buf_ld4b(r, vb, sb); }
  __device__ __forceinline__ void value2(const Raw2& v, float2& a, float2& b) const { unpack2(v, a, b); }
  __device__ __forceinline__ void own2(uint32_t i, float2* a, float2* b) const {
    unpack2(buf_ld4b(r, i * 8u, 0), a[0], b[0]);
  }
};
struct SrcBf16 {  // complex stored as a bf16 pair per element (not staged)
  __amdgpu_buffer_rsrc_t r;
  static constexpr int kNV = 1;
  static constexpr bool kStageable = false;
  static constexpr bool kPairs = false;
  using Raw = uint32_t;
  __device__ __forceinline__ Raw load(uint32_t i) const {
    return __builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, 0);
  }
  __device__ __forceinline__ Raw load_b(uint32_t vb, uint32_t sb) const {   // bytes of complex64
    return __builtin_amdgcn_raw_buffer_load_b32(r, vb >> 1, sb >> 1, 0);
  }
  __device__ __forceinline__ float2 value(Raw v) const { return bf16x2_to_f2(v); }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int) const { return r; }
  __device__ __forceinline__ float2 combine(const float2* v) const { return v[0]; }
  __device__ __forceinline__ void own(uint32_t i, float2* v) const { v[0] = value(load(i)); }
};
struct SrcDir {   // the new direction c + beta p, formed from c and the old p
  __amdgpu_buffer_rsrc_t c, p;
  float beta;
  static constexpr int kNV = 2;
  static constexpr bool kStageable = true;
  struct Raw {
    float2 c, p;
  };
  __device__ __forceinline__ Raw load(uint32_t i) const { return Raw{buf_ld2(c, i), buf_ld2(p, i)}; }
  __device__ __forceinline__ Raw load_b(uint32_t vb, uint32_t sb) const {
    return Raw{buf_ld2b(c, vb, sb), buf_ld2b(p, vb, sb)};
  }
  __device__ __forceinline__ float2 value(const Raw& v) const { return axpyf(beta, v.p, v.c); }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int j) const { return j == 0 ? c : p; }
  __device__ __forceinline__ float2 combine(const float2* v) const { return axpyf(beta, v[1], v[0]); }
  __device__ __forceinline__ void own(uint32_t i, float2* v) const {
    v[0] = buf_ld2(c, i);
    v[1] = buf_ld2(p, i);
  }
  static constexpr bool kPairs = true;
  struct Raw2 {
    u32x4 c, p;
  };
  __device__ __forceinline__ Raw2 load2_b(uint32_t vb, uint32_t sb) const {
    return Raw2{buf_ld4b(c, vb, sb), buf_ld4b(p, vb, sb)};
  }
  __device__ __forceinline__ void value2(const Raw2& v, float2& a, float2& b) const {
    float2 c0, c1, p0, p1;
    unpack2(v.c, c0, c1);
    unpack2(v.p, p0, p1);
    a = axpyf(beta, p0, c0);
    b = axpyf(beta, p1, c1);
  }
  __device__ __forceinline__ void own2(uint32_t i, float2* a, float2* b) const {
    unpack2(buf_ld4b(c, i * 8u, 0), a[0], b[0]);
    unpack2(buf_ld4b(p, i * 8u, 0), a[1], b[1]);
  }
};
struct SrcLds {   // complex64 vector in LDS
  LdsC v;
  using Raw = float2;
  __device__ __forceinline__ Raw load(uint32_t i) const { return v.ld((int)i); }
  __device__ __forceinline__ Raw load_b(uint32_t vb, uint32_t sb) const {
    return v.ld((int)((vb + sb) >> 3));
  }
  __device__ __forceinline__ float2 value(Raw x) const { return x; }
};

// Arithmetic of a band application: FP32 (the CG passes) or FP64 (the true-residual
// refresh), each with the delay-ramp and wrap tables of its precision.
struct ArithF32 {
  using C = float2;
  static constexpr uint32_t kTabBytes = 8;
  __device__ static __forceinline__ C zero() { return make_float2(0.f, 0.f); }
  __device__ static __forceinline__ C conj(C a) { return make_float2(a.x, -a.y); }
  __device__ static __forceinline__ C mul(C a, C b) { return cmulf(a, b); }
  __device__ static __forceinline__ void mac(C& acc, C c, C v) { cmacf(acc, c, v); }
  __device__ static __forceinline__ C from(float2 v) { return v; }
  __device__ static __forceinline__ const void* rtab(const FrameDev& F) { return F.rtab; }
  __device__ static __forceinline__ const void* wtab(const FrameDev& F) { return F.wtab; }
  __device__ static __forceinline__ C tab(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, vb, sb, 0));
  }
  __device__ static __forceinline__ C tab_s(const void* t, int i) {   // wave-uniform index
    return __builtin_bit_cast(float2, ((kptr<const u64>)t)[i]);
  }
  __device__ static __forceinline__ C tab_g(const void* t, int i) {
    return __builtin_bit_cast(float2, ((gptr<const u64>)t)[i]);
  }
};
struct ArithF64 {
  using C = double2;
  static constexpr uint32_t kTabBytes = 16;
  __device__ static __forceinline__ C zero() { return make_double2(0.0, 0.0); }
  __device__ static __forceinline__ C conj(C a) { return make_double2(a.x, -a.y); }
  __device__ static __forceinline__ C mul(C a, C b) { return cmuld(a, b); }
  __device__ static __forceinline__ void mac(C& acc, C c, C v) { cmacd(acc, c, v); }
  __device__ static __forceinline__ C from(float2 v) { return make_double2((double)v.x, (double)v.y); }
  __device__ static __forceinline__ C from(double2 v) { return v; }
  __device__ static __forceinline__ const void* rtab(const FrameDev& F) { return F.rtab64; }
  __device__ static __forceinline__ const void* wtab(const FrameDev& F) { return F.wtab64; }
  __device__ static __forceinline__ C tab(__amdgpu_buffer_rsrc_t r, uint32_t vb, uint32_t sb) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, vb, sb, 0));
  }
  __device__ static __forceinline__ C tab_s(const void* t, int i) {
    return __builtin_bit_cast(double2, ((kptr<const u32x4>)t)[i]);
  }
  __device__ static __forceinline__ C tab_g(const void* t, int i) {
    return __builtin_bit_cast(double2, ((gptr<const u32x4>)t)[i]);
  }
};
// The stored coefficient table D_{p,q} (Eq. D_definition, the SS table of Eq. ds_repr):
// one entry per (path, output element), P x E, as a bf16 pair or a complex64 value.
template <int SD>
struct DTab {   // kDNone: no table
  using Raw = uint32_t;
  const void* p;
  __device__ __forceinline__ Raw load(int64_t) const { return 0u; }
  __device__ __forceinline__ float2 value(Raw) const { return make_float2(0.f, 0.f); }
};
template <>
struct DTab<kDBf16> {
  using Raw = uint32_t;
  const void* p;
  __device__ __forceinline__ Raw load(int64_t i) const { return glb(static_cast<const uint32_t*>(p))[i]; }
  __device__ __forceinline__ float2 value(Raw w) const { return bf16x2_to_f2(w); }
};
template <>
struct DTab<kDC64> {
  using Raw = u64;
  const void* p;
  __device__ __forceinline__ Raw load(int64_t i) const { return glb(static_cast<const u64*>(p))[i]; }
  __device__ __forceinline__ float2 value(Raw w) const { return __builtin_bit_cast(float2, w); }
};

// A complex64 vector read and written element-wise through a buffer resource (one 32-bit
// offset per element, shared by every vector accessed at that element).
// NT: non-temporal cache policy (streamed data that should not displace gather sources
// in L2).
struct CVec {
  __amdgpu_buffer_rsrc_t r;
  template <bool NT = false>
  __device__ __forceinline__ float2 ld(uint32_t i) const {
    return __builtin_bit_cast(float2,
                              __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, NT ? 2 : 0));
  }
  template <bool NT = false>
  __device__ __forceinline__ void st(uint32_t i, float2 v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, i * 8u, 0,
                                          NT ? 2 : 0);
  }
  // elements i and i + 1 as one 16-byte access
  template <bool NT = false>
  __device__ __forceinline__ void ld2(uint32_t i, float2& a, float2& b) const {
    unpack2(buf_ld4b<NT ? 2 : 0>(r, i * 8u, 0), a, b);
  }
  template <bool NT = false>
  __device__ __forceinline__ void st2(uint32_t i, float2 a, float2 b) const {
    __builtin_amdgcn_raw_buffer_store_b128(pack2(a, b), r, i * 8u, 0, NT ? 2 : 0);
  }
};
#ifndef OTFS_NT
#define OTFS_NT 23
#endif
constexpr bool kNtElem = (OTFS_NT & 1) != 0;   // element-wise passes: loads
constexpr bool kNtElemSt = (OTFS_NT & 16) != 0;  // element-wise passes: x and c stored
constexpr bool kNtB = (OTFS_NT & 2) != 0;      // H^H pass: p' read, a stored
constexpr bool kNtT = (OTFS_NT & 4) != 0;      // H pass: t stored
constexpr bool kNtP = (OTFS_NT & 8) != 0;      // direction pass: p' stored
__device__ __forceinline__ CVec cvec(const float2* p, int64_t n) { return CVec{buf_rsrc(p, n * 8)}; }
__device__ __forceinline__ SrcBuf src_vec(const float2* p, int64_t n) {
  return SrcBuf{buf_rsrc(p, n * 8)};
}
__device__ __forceinline__ SrcDir src_dir(const float2* c, const float2* p, float beta,
                                          int64_t n) {
  return SrcDir{buf_rsrc(c, n * 8), buf_rsrc(p, n * 8), beta};
}

// Output views of a band application (see apply_band).
struct NoPre {};
// pre(q) / put(q, v, pre, own) handle output element q; pre2 / put2 the pair q, q + 1 of
// the paired gathers (q even), in the same operations per element.
template <bool NT = false>
struct OutStore {   // out = v
  CVec o;
  static constexpr bool kOwn = false;
  using Pre = NoPre;
  using Pre2 = NoPre;
  __device__ __forceinline__ Pre pre(uint32_t) const { return Pre{}; }
  __device__ __forceinline__ void put(uint32_t q, float2 v, const Pre&, const float2*) const {
    o.st<NT>(q, v);
  }
  __device__ __forceinline__ Pre2 pre2(uint32_t) const { return Pre2{}; }
  __device__ __forceinline__ void put2(uint32_t q, float2 v0, float2 v1, const Pre2&,
                                       const float2*, const float2*) const {
    o.st2<NT>(q, v0, v1);
  }
};
struct OutInit {    // b = H^H y: c = p = b, x = 0, partial ||b||^2
  CVec c, p, x;
  float* acc;
  static constexpr bool kOwn = false;
  using Pre = NoPre;
  __device__ __forceinline__ Pre pre(uint32_t) const { return Pre{}; }
  __device__ __forceinline__ void put(uint32_t q, float2 v, const Pre&, const float2*) const {
    c.st(q, v);
    p.st(q, v);
    x.st(q, make_float2(0.f, 0.f));
    *acc = fmaf(v.x, v.x, *acc);
    *acc = fmaf(v.y, v.y, *acc);
  }
  using Pre2 = NoPre;
  __device__ __forceinline__ Pre2 pre2(uint32_t) const { return Pre2{}; }
  __device__ __forceinline__ void put2(uint32_t q, float2 v0, float2 v1, const Pre2&,
                                       const float2*, const float2*) const {
    c.st2(q, v0, v1);
    p.st2(q, v0, v1);
    x.st2(q, make_float2(0.f, 0.f), make_float2(0.f, 0.f));
    *acc = fmaf(v0.x, v0.x, *acc);
    *acc = fmaf(v0.y, v0.y, *acc);
    *acc = fmaf(v1.x, v1.x, *acc);
    *acc = fmaf(v1.y, v1.y, *acc);
  }
};
struct OutA {       // t = H p', p_new = c + beta p_old, x += alpha p_old (deferred updates)
  CVec t, pn, x;
  float alpha, beta;
  bool xp;
  static constexpr bool kOwn = true;
  struct Pre {
    float2 x;
  };
  __device__ __forceinline__ Pre pre(uint32_t q) const {
    return Pre{xp ? x.ld(q) : make_float2(0.f, 0.f)};
  }
  __device__ __forceinline__ void put(uint32_t q, float2 v, const Pre& pr, const float2* own) const {
    t.st(q, v);   // default cache policy: measured faster here than the streamed one
    pn.st(q, axpyf(beta, own[1], own[0]));
    if (xp) x.st(q, axpyf(alpha, own[1], pr.x));
  }
  struct Pre2 {
    float2 x0, x1;
  };
  __device__ __forceinline__ Pre2 pre2(uint32_t q) const {
    Pre2 r{make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    if (xp) x.ld2(q, r.x0, r.x1);
    return r;
  }
  __device__ __forceinline__ void put2(uint32_t q, float2 v0, float2 v1, const Pre2& pr,
                                       const float2* own0, const float2* own1) const {
    t.st2(q, v0, v1);
    pn.st2(q, axpyf(beta, own0[1], own0[0]), axpyf(beta, own1[1], own1[0]));
    if (xp) x.st2(q, axpyf(alpha, own0[1], pr.x0), axpyf(alpha, own1[1], pr.x1));
  }
};
struct OutB {       // a = H^H t + lam p', partial Re(p'^H a)
  CVec a, pn;
  float lam;
  float* acc;
  static constexpr bool kOwn = false;
  struct Pre {
    float2 p;
  };
  __device__ __forceinline__ Pre pre(uint32_t q) const { return Pre{pn.ld<kNtB>(q)}; }
  __device__ __forceinline__ void put(uint32_t q, float2 v, const Pre& pr, const float2*) const {
    const float2 av = axpyf(lam, pr.p, v);
    a.st<kNtB>(q, av);
    *acc = fmaf(pr.p.x, av.x, *acc);
    *acc = fmaf(pr.p.y, av.y, *acc);
  }
  struct Pre2 {
    float2 p0, p1;
  };
  __device__ __forceinline__ Pre2 pre2(uint32_t q) const {
    Pre2 r;
    pn.ld2<kNtB>(q, r.p0, r.p1);
    return r;
  }
  __device__ __forceinline__ void put2(uint32_t q, float2 v0, float2 v1, const Pre2& pr,
                                       const float2*, const float2*) const {
    const float2 a0 = axpyf(lam, pr.p0, v0), a1 = axpyf(lam, pr.p1, v1);
    a.st2<kNtB>(q, a0, a1);
    *acc = fmaf(pr.p0.x, a0.x, *acc);
    *acc = fmaf(pr.p0.y, a0.y, *acc);
    *acc = fmaf(pr.p1.x, a1.x, *acc);
    *acc = fmaf(pr.p1.y, a1.y, *acc);
  }
};

// ---------------------------------------------------------------------------------------
// reductions: wave64 butterfly, then the waves of the block in a fixed order
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float block_sum(float v, float* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) s += red[i];
  __syncthreads();
  return s;
}
__device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum_d(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) s += red[i];
  __syncthreads();
  return s;
}
// sum of the T per-tile partials of a frame, in FP32 and in tile order, by every thread:
// every workgroup of the frame forms the same value, independent of the rest of the batch
__device__ __forceinline__ float tile_sum(const float* part, int T) {
  // loads in groups of 8 in flight together; the sum runs in tile order
  float s = 0.f;
  int i = 0;
  for (; i + 8 <= T; i += 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[i + j];
#pragma unroll
    for (int j = 0; j < 8; ++j) s = __fadd_rn(s, v[j]);
  }
  for (; i < T; ++i) s = __fadd_rn(s, part[i]);
  return s;
}
__device__ __forceinline__ double tile_sum_d(const double* part, int T) {
  double s = 0.0;
  int i = 0;
  for (; i + 8 <= T; i += 8) {
    double v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[i + j];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  for (; i < T; ++i) s += part[i];
  return s;
}

// ---------------------------------------------------------------------------------------
// per-frame barrier among the T workgroups that share a frame
// ---------------------------------------------------------------------------------------
// Two coherence modes.
//  XCD-local (all workgroups of the frame run on one XCD, whose L2 they share): every
//  thread waits for its own stores to reach the L2 (s_waitcnt vmcnt(0); no L2 write-back,
//  so the data stays in the shared L2), one lane counts the arrival with an L2 atomic and
//  polls the count with L2 atomics, and after the workgroup meets again every thread
//  takes an agent-scope acquire (buffer_inv sc1), which drops this CU's L1.  The
//  workgroup-scope invalidate (buffer_inv sc0) is not enough: outside threadgroup-split
//  mode it leaves L1 lines written by other CUs stale (measured).
//  Agent (fallback, any placement): agent-scope release and acquire fences (L2 write-back
//  and invalidate, the L2s of different XCDs not being coherent) around an agent-scope
//  counter.
// The wait is bounded: after `timeout` ticks of the 100 MHz wall clock, or when another
// workgroup has raised the launch-wide abort flag, it gives up and reports failure.
__device__ __forceinline__ void xcd_release() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void xcd_acquire() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Current value of a counter kept in the L2 by workgroup-scope atomics.  A plain or
// idempotent read could be served by this CU's L1 (the compiler turns an idempotent RMW
// such as fetch_add(0) into a load), so the poll is a compare-and-swap whose compare
// value the counter never holds: it always executes in the L2 and never writes.
__device__ __forceinline__ unsigned l2_poll(unsigned* ctr) {
  unsigned expected = 0xffffffffu;
  __hip_atomic_compare_exchange_strong(ctr, &expected, 0xfffffffeu, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return expected;
}

__device__ bool frame_barrier(unsigned* ctr, unsigned target, bool xcd_local,
                              unsigned* abort_flag, uint64_t timeout, int* sflag) {
  if (xcd_local)
    xcd_release();
  else
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    if (xcd_local) {
      unsigned v = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) + 1u;
      while (v < target) {
        __builtin_amdgcn_s_sleep(1);
        v = l2_poll(ctr);
        if (v >= target) break;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > timeout) {
          __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    } else {
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > timeout) {
          __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    *sflag = ok;
  }
  __syncthreads();
  if (xcd_local)
    xcd_acquire();
  else
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *sflag != 0;
}

// Neighbour synchronisation.  Between the direction pass and the H pass, and between the
// H pass and the H^H pass, a tile reads only rows within the Doppler shift range of its
// own band, so it waits for the tiles owning those rows instead of the whole frame.  Each
// tile counts the phases it has finished in prog[tile] (an L2 atomic after its stores are
// released); a waiting tile polls the counters of the tiles it reads, one lane per tile.
// Every earlier writer of the rows it reads is separated from the read by a full barrier.
__device__ __forceinline__ void tile_publish(unsigned* flag, bool xcd_local) {
  if (xcd_local)
    xcd_release();
  else
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(flag, 1u, __ATOMIC_RELAXED,
                           xcd_local ? __HIP_MEMORY_SCOPE_WORKGROUP : __HIP_MEMORY_SCOPE_AGENT);
}

// Tiles owning the cyclic row range [r0, r0 + span) of a frame of N rows in T bands
// (band t = [t N / T, (t + 1) N / T)): first tile and count.
struct TileRange {
  int first, count;
};
__device__ __forceinline__ int tile_of_row(int r, int N, int T) {
  return (int)((((int64_t)r + 1) * T - 1) / N);
}
__device__ __forceinline__ TileRange tiles_of_rows(int r0, int span, int N, int T) {
  if (span >= N) return TileRange{0, T};
  r0 %= N;
  if (r0 < 0) r0 += N;
  int r1 = r0 + span - 1;
  if (r1 >= N) r1 -= N;
  const int t0 = tile_of_row(r0, N, T), t1 = tile_of_row(r1, N, T);
  int cnt = t1 - t0 + 1;
  if (cnt <= 0) cnt += T;
  return TileRange{t0, cnt};
}

__device__ bool halo_wait(const unsigned* prog, int T, TileRange tr, unsigned target,
                          bool xcd_local, unsigned* abort_flag, uint64_t timeout, int* sflag) {
  if (threadIdx.x < 64) {
    const int lane = (int)threadIdx.x;
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    for (int b = 0; b < tr.count && ok; b += 64) {
      const int j = b + lane;
      bool done = j >= tr.count;
      int tile = tr.first + j;
      if (tile >= T) tile -= T;
      unsigned* fl = const_cast<unsigned*>(prog) + (done ? 0 : tile);
      for (;;) {
        if (!done) {
          const unsigned v = xcd_local ? l2_poll(fl)
                                       : __hip_atomic_load(fl, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
          done = v >= target;
        }
        if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            wall_clock64() - t0 > timeout) {
          if (lane == 0)
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (lane == 0) *sflag = ok;
  }
  __syncthreads();
  if (xcd_local)
    xcd_acquire();
  else
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *sflag != 0;
}

// ---------------------------------------------------------------------------------------
// Band application of H (ADJ = false) or H^H (ADJ = true).
//
// A workgroup owns Doppler rows [lb, le) of one frame.  Thread (tx, ty) walks delay
// columns k = tx, tx + TX, ... and, for each, the rows lb + ty + i*TY of the band in
// chunks of R rows.  For one chunk the loop runs over the paths: the chunk's R gathers of
// path p are independent loads issued together (R loads in flight per lane), each a
// contiguous run of a source row across the wave, and the coefficient of the column is
// loaded once per (chunk, path).  Nothing is sized by P, so one kernel serves every P.
//
// src is a source view (see SrcBuf): src.load(i) issues the reads of element i (frame-local
// index) of the vector being multiplied and src.value(raw) forms the element; every read
// of a chunk is issued before the first value is formed, and no read sits under a
// branch, so the R*U gathers of a chunk are in flight together.  Rows past the end of the
// band repeat the band's last row and are not stored.  sink(q, v) receives output element
// q.  Threads without a column return early; callers put block-wide work after the call.
//
// Wrap factor.  W[l0]^n with l0 the source row: for H, l0 = <l - nu>_N and
// W[l0] = W[l] conj(W[nu]), so the path part conj(W[nu])^n is folded into the column's
// coefficient and only W[l]^n (one table read per row of the chunk) varies along the
// band; for H^H the factor is W[l]^w of the output row itself.
// ---------------------------------------------------------------------------------------
#ifndef OTFS_ROWS
#define OTFS_ROWS 4
#endif
#ifndef OTFS_PATHS
#define OTFS_PATHS 4
#endif
#ifndef OTFS_STRIP_LANES
#define OTFS_STRIP_LANES 64
#endif
// Lanes across one row in the gather passes (a multiple of 64): a band is walked in
// strips of that many delay columns (twice as many in the paired form), every row of the
// band per strip, so the source rows a strip reaches stay in cache while its paths reuse
// them.
constexpr int kStripLanes = OTFS_STRIP_LANES;
// Lanes across a row for a band of band_rows rows walked R rows per thread chunk: the
// strip width, widened (doubling, up to a whole workgroup) while the band is too short to
// give every thread R rows; at most `width` (the lanes a whole row needs).  Wave-uniform.
__device__ __forceinline__ int strip_lanes(int width, int band_rows, int R) {
  int t = kStripLanes;
  while (t < kBlock && t * band_rows < kBlock * R) t <<= 1;
  return width < t ? width : t;
}
constexpr int kRows = OTFS_ROWS;    // rows per thread chunk in the FP32 gathers
constexpr int kPaths = OTFS_PATHS;  // paths whose gathers are in flight together
static_assert(kRows == OTFS_ROWS, "the host's strip rule assumes kRows rows per chunk");
#ifndef OTFS_PATHS_GENERAL
#define OTFS_PATHS_GENERAL 2
#endif
constexpr int kPathsGeneral = OTFS_PATHS_GENERAL;   // the same where rows are per lane
#ifndef OTFS_FD_ROWS
#define OTFS_FD_ROWS 4
#endif
#ifndef OTFS_FD_PATHS
#define OTFS_FD_PATHS 1
#endif
constexpr int kFdRows = OTFS_FD_ROWS;     // H pass forming the direction in its gathers
constexpr int kFdPaths = OTFS_FD_PATHS;
#ifndef OTFS_PAIR_PATHS
#define OTFS_PAIR_PATHS 4
#endif
// paths in flight together in the paired gathers (each gather holds twice the registers)
constexpr int kPairPaths = OTFS_PAIR_PATHS;
#ifndef OTFS_FUSED_MIN_WAVES
#define OTFS_FUSED_MIN_WAVES 2
#endif
#ifndef OTFS_ELEM_CHUNK
#define OTFS_ELEM_CHUNK 8
#endif
constexpr int kElemChunk = OTFS_ELEM_CHUNK;   // elements per thread in flight, element-wise passes
#ifndef OTFS_ELEM_CHUNK_FD
#define OTFS_ELEM_CHUNK_FD 16
#endif
constexpr int kElemChunkFd = OTFS_ELEM_CHUNK_FD;   // the same in the direct-fd kind (more registers free)
#ifndef OTFS_ELEM_CHUNK_LDS
#define OTFS_ELEM_CHUNK_LDS 16
#endif
constexpr int kElemChunkLds = OTFS_ELEM_CHUNK_LDS;   // and in the windowed-pairs kind
#ifndef OTFS_RES_ROWS
#define OTFS_RES_ROWS 2
#endif
#ifndef OTFS_RES_PATHS
#define OTFS_RES_PATHS 1
#endif
constexpr int kResRows = OTFS_RES_ROWS;    // rows per chunk of the LDS-resident gathers
constexpr int kResPaths = OTFS_RES_PATHS;  // paths per step of the LDS-resident gathers

template <int R, int U, bool ADJ, int SD, bool UNI, class A, class Src, class Pref, class Sink>
__device__ __forceinline__ void band_apply_rows(const FrameDev& F, int lb, int le, const Src& src,
                                                Pref pref, Sink sink) {
  using C = typename A::C;
  constexpr bool STORED = SD != kDNone;
  const int M = F.M, N = F.N, P = F.P;
  const int TX = strip_lanes(M, le - lb, R);
  const int TY = kBlock / TX;
  const int tx = threadIdx.x % TX;
  // UNI: TX is a multiple of 64, so every wave lies in one row group ty and the row
  // arithmetic below is the same for all its lanes (scalar registers, scalar offsets).
  const int ty = UNI ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / TX)
                     : (int)threadIdx.x / TX;
  if (ty >= TY) return;
  const int64_t E = (int64_t)M * N;
  const uint32_t M8 = 8u * (uint32_t)M, E8 = 8u * (uint32_t)E;   // E8 < 2^31
  constexpr uint32_t TS = A::kTabBytes / 8u;                      // table entry / 8 bytes
  const int nrows = le - lb - ty > 0 ? (le - lb - ty + TY - 1) / TY : 0;
  const KPairs paths = kpairs(F.paths);
  const void* wt = A::wtab(F);
  const __amdgpu_buffer_rsrc_t rtab = buf_rsrc(A::rtab(F), (int64_t)P * M * A::kTabBytes);
  const DTab<SD> dtab{F.dtab};
  for (int k = tx; k < M; k += TX) {
    for (int r0 = 0; r0 < nrows; r0 += R) {
      int l[R];
      uint32_t l8[R];   // byte offset of row l
      C wl[R];
      C acc[R];
      decltype(pref(0u)) pf[R];   // the outputs' own loads, issued with the gathers
#pragma unroll
      for (int i = 0; i < R; ++i) {
        l[i] = lb + ty + min(r0 + i, nrows - 1) * TY;
        l8[i] = (uint32_t)l[i] * M8;
        if (!STORED) wl[i] = UNI ? A::tab_s(wt, l[i]) : A::tab_g(wt, l[i]);
        acc[i] = A::zero();
        pf[i] = pref((uint32_t)(l[i] * M + k));
      }
      // NP paths at once: all NP*R gathers are issued before any is consumed
      auto step = [&](auto npc, int p0) {
        constexpr int NP = decltype(npc)::value;
        uint32_t kk8[NP], dn8[NP];
        bool lo[NP], hi[NP];   // delay wrap: the source column is K + M (lo) or K - M (hi)
        C cf[NP], wn[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          const int2 tn = paths.i2(p0 + u);
          const int K = ADJ ? k + tn.x : k - tn.x;   // H: <k - tau>_M; H^H: <k + tau>_M
          lo[u] = K < 0;
          hi[u] = K >= M;
          kk8[u] = 8u * (uint32_t)(lo[u] ? K + M : (hi[u] ? K - M : K));
          // source row <l -+ nu>_N = l + d - N (+ N when negative), d = <-+nu>_N
          const int sh = ADJ ? tn.y : -tn.y;
          dn8[u] = (uint32_t)((sh < 0 ? sh : sh - N) * M8);
          if (!STORED) {
            const C r = A::tab(rtab, TS * (ADJ ? kk8[u] : 8u * (uint32_t)k),
                               TS * (uint32_t)(p0 + u) * M8);
            cf[u] = ADJ ? A::conj(r) : r;
            if (!ADJ) wn[u] = A::tab_s(wt, tn.y < 0 ? tn.y + N : tn.y);
          }
        }
        typename Src::Raw v[NP][R];
        typename DTab<SD>::Raw d[NP][R];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
#pragma unroll
          for (int i = 0; i < R; ++i) {
            // (ls - N) * 8M wraps below zero exactly when ls < N; min picks the row in range
            const uint32_t x = l8[i] + dn8[u];
            const uint32_t rs = min(x, x + E8);
            if (UNI)
              v[u][i] = src.load_b(kk8[u], rs);
            else
              v[u][i] = src.load_b(kk8[u] + rs, 0u);
            if (STORED)
              d[u][i] = dtab.load((int64_t)(p0 + u) * E +
                                  (ADJ ? (int64_t)((rs + kk8[u]) >> 3) : (int64_t)l[i] * M + k));
          }
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          if constexpr (STORED) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
              const float2 dd = dtab.value(d[u][i]);
              A::mac(acc[i], ADJ ? A::conj(dd) : dd, A::from(src.value(v[u][i])));
            }
          } else {
            if (__builtin_amdgcn_ballot_w64(lo[u] || hi[u]) != 0) {
              // a wave holding a delay wrap of this path (few of them): wrapped lanes take
              // W^n, n = -1 (lo) or +1 (hi); for H also the path part conj(W[nu])^n
              C cw = cf[u];
              if (!ADJ) {
                C wv = wn[u];
                if (hi[u]) wv.y = -wv.y;
                cw = A::mul(cf[u], wv);
              }
#pragma unroll
              for (int i = 0; i < R; ++i) {
                C w = wl[i];
                if (!hi[u]) w.y = -w.y;
                const C c = (lo[u] || hi[u]) ? A::mul(cw, w) : cf[u];
                A::mac(acc[i], c, A::from(src.value(v[u][i])));
              }
            } else {
#pragma unroll
              for (int i = 0; i < R; ++i) A::mac(acc[i], cf[u], A::from(src.value(v[u][i])));
            }
          }
        }
      };
      int p = 0;
      for (; p + U <= P; p += U) step(std::integral_constant<int, U>{}, p);
      if constexpr (U > 2) {
        if (p + 2 <= P) {
          step(std::integral_constant<int, 2>{}, p);
          p += 2;
        }
      }
      for (; p < P; ++p) step(std::integral_constant<int, 1>{}, p);
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (r0 + i < nrows) sink(l[i] * M + k, acc[i], pf[i]);
    }
  }
}

template <int R, int U, bool ADJ, int SD, class Src, class Pref, class Sink, class A = ArithF32>
__device__ __forceinline__ void band_apply(const FrameDev& F, int lb, int le, const Src& src,
                                           Pref pref, Sink sink, A = A{}) {
  const int TX = strip_lanes(F.M, le - lb, R);
  // the per-lane row arithmetic of the general form holds more registers: fewer paths
  // in flight there
  if ((TX & 63) == 0)
    band_apply_rows<R, U, ADJ, SD, true, A>(F, lb, le, src, pref, sink);
  else
    band_apply_rows<R, (U < kPathsGeneral ? U : kPathsGeneral), ADJ, SD, false, A>(F, lb, le, src,
                                                                                     pref, sink);
}

// Frames whose gathers run in pairs: M a multiple of 128 (every wave in one row), and the
// frame at an even element offset in batch-wide buffers (16-byte aligned pairs).
__device__ __forceinline__ bool pairs_ok(const FrameDev& F) {
#ifdef OTFS_NO_PAIRS
  return false;
#else
  return (F.M & 127) == 0 && (F.off & 1) == 0;
#endif
}

// ---------------------------------------------------------------------------------------
// Paired band application (frames with M a multiple of 128, synthesised coefficients).
//
// The same sums as band_apply_rows, but each lane owns two adjacent delay columns k, k + 1
// (k even) and every access moves 16 bytes: one gather brings the two source elements
// <k -+ tau>_M and <k + 1 -+ tau>_M of a row, one table read the two coefficients of H
// (R_p[k], R_p[k + 1]), one store the two outputs.  A wave reads or writes 1 KiB per
// instruction instead of 512 B, which halves the vector-memory instructions for the same
// bytes (the gathers are bound by the rate at which those instructions issue, not by the
// bytes they move).  The one lane of a row whose two sources straddle the row's wrap point
// (source columns M - 1 and 0, or for H^H coefficients R_p[M - 1] and R_p[0]) takes its
// second element from a fix-up read at column 0, issued only by the waves holding such a
// lane, together with the main reads.  Wrap factors apply per element exactly as in
// band_apply_rows (each element has its own wrap count), so each output element is formed
// by the same operations in the same path order.
// ---------------------------------------------------------------------------------------
template <int R, int U, bool ADJ, class Src, class Pref, class Sink>
__device__ __forceinline__ void band_apply_pairs(const FrameDev& F, int lb, int le, const Src& src,
                                                 Pref pref, Sink sink) {
  const int M = F.M, N = F.N, P = F.P;
  const int M2 = M >> 1;
  const int TX = strip_lanes(M2, le - lb, R);   // a multiple of 64: waves in one row
  const int TY = kBlock / TX;
  const int tx = threadIdx.x % TX;
  const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TX);
  if (ty >= TY) return;
  const int64_t E = (int64_t)M * N;
  const uint32_t M8 = 8u * (uint32_t)M, E8 = 8u * (uint32_t)E;   // E8 < 2^31
  const int nrows = le - lb - ty > 0 ? (le - lb - ty + TY - 1) / TY : 0;
  const KPairs paths = kpairs(F.paths);
  const KPairs wtab_s = kpairs(F.wtab);
  const __amdgpu_buffer_rsrc_t rtab = buf_rsrc(F.rtab, (int64_t)P * M * 8);
  for (int k = 2 * tx; k < M; k += 2 * TX) {
    // Whether a pair of this strip of columns can wrap around the delay axis (or straddle
    // the row's wrap point) for a path in the frame's delay range: uniform over the strip.
    // Strips that cannot run a row loop without the wrap and fix-up branches, whose
    // accumulators then stay in place; the per-pair tests decide as before elsewhere.
    const int k0 = k - 2 * tx, kmax = min(k0 + 2 * TX, M) - 2;
    const int kmin_src = ADJ ? k0 + F.tau_lo : k0 - F.tau_hi;
    const int kmax_src = ADJ ? kmax + F.tau_hi : kmax - F.tau_lo;
    const bool strip_wraps = kmin_src < 0 || kmax_src + 1 >= M;
    auto rows = [&](auto wrap_c) __attribute__((always_inline)) {
    constexpr bool WRAP = decltype(wrap_c)::value;
    for (int r0 = 0; r0 < nrows; r0 += R) {
      int l[R];
      uint32_t l8[R];
      float2 wl[R];
      float2 acc0[R], acc1[R];
      decltype(pref(0u)) pf[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        l[i] = lb + ty + min(r0 + i, nrows - 1) * TY;
        l8[i] = (uint32_t)l[i] * M8;
        wl[i] = wtab_s.f(l[i]);
        acc0[i] = make_float2(0.f, 0.f);
        acc1[i] = make_float2(0.f, 0.f);
        pf[i] = pref((uint32_t)(l[i] * M + k));
      }
      auto step = [&](auto npc, int p0) {
        constexpr int NP = decltype(npc)::value;
        uint32_t kk8[NP], dn8[NP];
        bool lo0[NP], hi0[NP], lo1[NP], hi1[NP], split[NP];
        u32x4 cf2[NP];
        float2 wn[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          const int2 tn = paths.i2(p0 + u);
          const int K = ADJ ? k + tn.x : k - tn.x;   // source column of element 0 (unwrapped)
          lo0[u] = K < 0;
          hi0[u] = K >= M;
          lo1[u] = K + 1 < 0;
          hi1[u] = K + 1 >= M;
          const int s0 = lo0[u] ? K + M : (hi0[u] ? K - M : K);
          split[u] = s0 == M - 1;
          kk8[u] = 8u * (uint32_t)s0;
          const int sh = ADJ ? tn.y : -tn.y;
          dn8[u] = (uint32_t)((sh < 0 ? sh : sh - N) * M8);
          // H: R_p[k], R_p[k + 1]; H^H: R_p at the two source columns (conjugated below)
          cf2[u] = buf_ld4b(rtab, ADJ ? kk8[u] : 8u * (uint32_t)k, (uint32_t)(p0 + u) * M8);
          if (!ADJ) wn[u] = wtab_s.f(tn.y < 0 ? tn.y + N : tn.y);
        }
        typename Src::Raw2 v[NP][R];
        typename Src::Raw fx[NP][R];   // fix-up: second element of a straddling pair
        float2 cfx[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const uint32_t x = l8[i] + dn8[u];
            const uint32_t rs = min(x, x + E8);
            v[u][i] = src.load2_b(kk8[u], rs);
          }
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          if (WRAP && __builtin_amdgcn_ballot_w64(split[u]) != 0) {
#pragma unroll
            for (int i = 0; i < R; ++i) {
              const uint32_t x = l8[i] + dn8[u];
              const uint32_t rs = min(x, x + E8);
              fx[u][i] = src.load_b(0u, rs);
            }
            if (ADJ) cfx[u] = __builtin_bit_cast(
                float2, __builtin_amdgcn_raw_buffer_load_b64(rtab, 0u, (uint32_t)(p0 + u) * M8, 0));
          }
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          float2 c0, c1;
          unpack2(cf2[u], c0, c1);
          const bool sp = WRAP && __builtin_amdgcn_ballot_w64(split[u]) != 0;
          if (ADJ) {
            if (sp && split[u]) c1 = cfx[u];
            c0 = make_float2(c0.x, -c0.y);
            c1 = make_float2(c1.x, -c1.y);
          }
          float2 e0[R], e1[R];
#pragma unroll
          for (int i = 0; i < R; ++i) {
            src.value2(v[u][i], e0[i], e1[i]);
            if (sp && split[u]) e1[i] = src.value(fx[u][i]);
          }
          if (WRAP && __builtin_amdgcn_ballot_w64(lo0[u] || hi0[u] || lo1[u] || hi1[u]) != 0) {
            // waves holding a delay wrap of this path: wrapped elements take W^n
            float2 cw0 = c0, cw1 = c1;
            if (!ADJ) {
              cw0 = cmulf(c0, make_float2(wn[u].x, hi0[u] ? -wn[u].y : wn[u].y));
              cw1 = cmulf(c1, make_float2(wn[u].x, hi1[u] ? -wn[u].y : wn[u].y));
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
              const float2 w0 = make_float2(wl[i].x, hi0[u] ? wl[i].y : -wl[i].y);
              const float2 w1 = make_float2(wl[i].x, hi1[u] ? wl[i].y : -wl[i].y);
              cmacf(acc0[i], (lo0[u] || hi0[u]) ? cmulf(cw0, w0) : c0, e0[i]);
              cmacf(acc1[i], (lo1[u] || hi1[u]) ? cmulf(cw1, w1) : c1, e1[i]);
            }
          } else {
#pragma unroll
            for (int i = 0; i < R; ++i) {
              cmacf(acc0[i], c0, e0[i]);
              cmacf(acc1[i], c1, e1[i]);
            }
          }
        }
      };
      int p = 0;
      for (; p + U <= P; p += U) step(std::integral_constant<int, U>{}, p);
      if constexpr (U > 2) {
        if (p + 2 <= P) {
          step(std::integral_constant<int, 2>{}, p);
          p += 2;
        }
      }
      for (; p < P; ++p) step(std::integral_constant<int, 1>{}, p);
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (r0 + i < nrows) sink((uint32_t)(l[i] * M + k), acc0[i], acc1[i], pf[i]);
    }
    };
    if (strip_wraps)
      rows(std::true_type{});
    else
      rows(std::false_type{});
  }
}

// ---------------------------------------------------------------------------------------
// LDS-windowed paired band application (frames of the staged kind with F.lpk > 0).
//
// The outputs, their assignment to threads, the order in which each thread produces them
// and the operations forming each one are those of band_apply_pairs, so the two give
// identical bits; only where the source elements come from changes.  For each strip of
// KC = 2 TX delay columns (TX lanes across a row, as band_apply_pairs chooses them) the
// workgroup first copies the strip's source window -- every row the band's paths reach
// (rows [lb - nu_hi, le - nu_lo) for H, [lb + nu_lo, le + nu_hi) for H^H, or all N) times
// F.lwc columns from an even column origin (or all M columns and the first two again) --
// into LDS with 16-byte direct-to-LDS loads (buffer_load_dwordx4 ... lds: a wave fills 1 KiB,
// 128 consecutive window elements, each lane two elements of one row), then every path's
// gathers read the window: an element is fetched from memory once per strip instead of
// once per path.  Window element (r, c) holds the source at row <row0 + r>_N, column
// <col0 + c>_M, so a pair whose two sources straddle the row's wrap point is adjacent in
// the window and needs no fix-up read.  The H^H coefficients R_p at the source columns
// still come from the table in memory (with the fix-up for a straddling pair).
// ---------------------------------------------------------------------------------------
constexpr int kLdsRows = 8;   // output rows per thread chunk in the LDS-windowed gathers

// Whether band [lb, le)'s window fits the frame's LDS window geometry (F.lwr x F.lwc) with
// its current shift ranges (a path table made on the device may widen them).
__device__ __forceinline__ bool lds_window_fits(const FrameDev& F, int lb, int le) {
  const int band = le - lb, dnu = F.nu_hi - F.nu_lo;
  const int wr = band + dnu >= F.N ? F.N : band + dnu;
  if (wr > F.lwr) return false;
  if (F.lwc >= F.M) return true;
  int wc = 2 * strip_lanes(F.M >> 1, band, kRows) + (F.tau_hi - F.tau_lo) + 1;
  wc += wc & 1;
  return wc < F.M && wc <= F.lwc;
}

template <class C>
__device__ __forceinline__ C cplx(decltype(C{}.x) x, decltype(C{}.x) y) {
  return C{x, y};
}

// A: the arithmetic (ArithF32 for the CG passes; ArithF64 for the true-residual refresh,
// whose sums and coefficients are FP64 while the window holds the FP32 source).
template <bool ADJ, class A, class Pref, class Sink>
__device__ __forceinline__ void lds_apply_pairs(const FrameDev& F, int lb, int le, const SrcBuf& src,
                                                float2* lds_gen, Pref pref, Sink sink, A = A{}) {
  using C = typename A::C;
  constexpr bool F32 = std::is_same<A, ArithF32>::value;
  constexpr uint32_t TS = A::kTabBytes / 8u;   // table entry / 8 bytes
  const int M = F.M, N = F.N, P = F.P;
  const int TX = strip_lanes(M >> 1, le - lb, kRows);   // band_apply_pairs's strip width
  const int TY = kBlock / TX;
  const int tx = threadIdx.x % TX;
  const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TX);
  const bool act = ty < TY;
  const int KC = 2 * TX;
  const int nrows = (act && le - lb - ty > 0) ? (le - lb - ty + TY - 1) / TY : 0;
  const int band = le - lb, dnu = F.nu_hi - F.nu_lo;
  const bool full_rows = band + dnu >= N;
  const int WR = full_rows ? N : band + dnu;
  const int row0 = full_rows ? 0 : (ADJ ? lb + F.nu_lo : lb - F.nu_hi);
  const int WC = F.lwc;                  // even; M + 2 when the window spans every column
  const bool full_cols = WC >= M;
  const int total = WR * WC;
  const int nchunk = (total + 127) >> 7;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const uint32_t M8 = 8u * (uint32_t)M;
  const KPairs paths = kpairs(F.paths);
  const void* wt = A::wtab(F);
  const __amdgpu_buffer_rsrc_t rtab = buf_rsrc(A::rtab(F), (int64_t)P * M * A::kTabBytes);
  const lptr<u64> win = (lptr<u64>)lds_gen;
  // A wave's window chunks are kWaves * 128 elements apart: its lane's (row, column) in the
  // window advances by (dr, dc) from one chunk to the next, so the walk needs no division.
  const int dr = (kWaves << 7) / WC, dc = (kWaves << 7) - dr * WC;   // dc < WC
  const int e_lane = (wave << 7) + 2 * lane;
  const int r_lane = e_lane / WC, c_lane = e_lane - r_lane * WC;
  for (int k0 = 0; k0 < M; k0 += KC) {
    const int col0 = full_cols ? 0 : ((ADJ ? k0 + F.tau_lo : k0 - F.tau_hi) & ~1);
    __syncthreads();   // the previous strip's window is no longer read
    int e = e_lane, r = r_lane, cc = c_lane;
    for (int c = wave; c < nchunk; c += kWaves) {
      if (e < total) {
        int sr = row0 + r;
        sr += sr < 0 ? N : 0;
        sr -= sr >= N ? N : 0;
        int sc = col0 + cc;
        sc += sc < 0 ? M : 0;
        sc -= sc >= M ? M : 0;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(src.r, (lptr<void>)(win + (c << 7)), 16,
                                                 (uint32_t)(sr * M + sc) * 8u, 0, 0, 0);
      }
      e += kWaves << 7;
      r += dr;
      cc += dc;
      if (cc >= WC) {
        cc -= WC;
        ++r;
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    const int k = k0 + 2 * tx;
    if (nrows == 0 || k >= M) continue;
    // Whether any pair of this strip wraps around the delay axis for a path in the frame's
    // delay range (uniform over the strip; the per-pair tests below then decide as before).
    // Strips that do not, in a band window, run a chunk loop with neither the wrap branch
    // nor the row wrap: its accumulators stay in place (no copies between the branches).
    const int kmax = min(k0 + KC, M) - 2;
    const int kmin_src = ADJ ? k0 + F.tau_lo : k0 - F.tau_hi;
    const int kmax_src = ADJ ? kmax + F.tau_hi : kmax - F.tau_lo;
    const bool strip_wraps = kmin_src < 0 || kmax_src + 1 >= M;
    auto chunks = [&](auto wrap_c, auto rows_c) __attribute__((always_inline)) {
    constexpr bool WRAP = decltype(wrap_c)::value;
    constexpr int FR = decltype(rows_c)::value;   // 0: band window, 1: all rows, 2: either
    for (int j0 = 0; j0 < nrows; j0 += kLdsRows) {
      int l[kLdsRows];
      C wl[kLdsRows];
      C acc0[kLdsRows], acc1[kLdsRows];
      decltype(pref(0u)) pf[kLdsRows];
#pragma unroll
      for (int i = 0; i < kLdsRows; ++i) {
        l[i] = lb + ty + min(j0 + i, nrows - 1) * TY;
        wl[i] = A::tab_s(wt, l[i]);
        acc0[i] = A::zero();
        acc1[i] = A::zero();
        pf[i] = pref((uint32_t)(l[i] * M + k));
      }
      // window row of output row i for a path with Doppler shift sh
      auto wrow = [&](int i, int sh) __attribute__((always_inline)) {
        int lr = l[i] + sh;
        if (FR == 1 || (FR == 2 && full_rows)) {
          lr += lr < 0 ? N : 0;
          lr -= lr >= N ? N : 0;
        } else {
          lr -= row0;
        }
        return lr;
      };
      // the pairs of the kLdsRows rows for one path: every LDS read is issued before any
      // is used (the FP64 form would otherwise convert each pair as it arrives and wait
      // for the reads one at a time)
      auto window_reads = [&](C* e0, C* e1, auto addr) __attribute__((always_inline)) {
        float2 r0[kLdsRows], r1[kLdsRows];
#pragma unroll
        for (int i = 0; i < kLdsRows; ++i) {
          const lptr<u64> w = addr(i);
          r0[i] = __builtin_bit_cast(float2, w[0]);
          r1[i] = __builtin_bit_cast(float2, w[1]);
        }
        if constexpr (!F32) asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < kLdsRows; ++i) {
          e0[i] = A::from(r0[i]);
          e1[i] = A::from(r1[i]);
        }
      };
      if constexpr (!WRAP) {
        // No pair of the strip wraps: every source column is K = k -+ tau in [0, M - 2].
        // The coefficients of the next path are requested before the current one is
        // applied, so their latency overlaps its LDS reads and products (same values, same
        // order); two register sets alternate, so nothing waits on a copy.
        struct Cf {
          C c0, c1;
        };
        auto coef = [&](int p, int2& tn) __attribute__((always_inline)) {
          tn = paths.i2(p);
          const uint32_t kc = ADJ ? (uint32_t)(k + tn.x) : (uint32_t)k;
          Cf r;
          if constexpr (F32) {
            float2 f0, f1;
            unpack2(buf_ld4b(rtab, 8u * kc, (uint32_t)p * M8), f0, f1);
            r.c0 = A::from(f0);
            r.c1 = A::from(f1);
          } else {   // one 16-byte entry per column
            r.c0 = A::tab(rtab, TS * 8u * kc, TS * (uint32_t)p * M8);
            r.c1 = A::tab(rtab, TS * 8u * (kc + 1u), TS * (uint32_t)p * M8);
          }
          return r;
        };
        auto apply = [&](int2 tn, const Cf& cf) __attribute__((always_inline)) {
          C c0 = cf.c0, c1 = cf.c1;
          if (ADJ) {
            c0 = A::conj(c0);
            c1 = A::conj(c1);
          }
          const int K = ADJ ? k + tn.x : k - tn.x;
          const int lc = full_cols ? K : K - col0;
          const int sh = ADJ ? tn.y : -tn.y;
          C e0[kLdsRows], e1[kLdsRows];
          window_reads(e0, e1, [&](int i) { return win + wrow(i, sh) * WC + lc; });
#pragma unroll
          for (int i = 0; i < kLdsRows; ++i) {
            A::mac(acc0[i], c0, e0[i]);
            A::mac(acc1[i], c1, e1[i]);
          }
        };
        int2 ta, tb;
        Cf ca = coef(0, ta);
        int p = 0;
        for (; p + 1 < P; p += 2) {
          const Cf cb = coef(p + 1, tb);
          apply(ta, ca);
          ca = coef(p + 2 < P ? p + 2 : p + 1, ta);
          apply(tb, cb);
        }
        if (p < P) apply(ta, ca);
      } else
      for (int p = 0; p < P; ++p) {
        const int2 tn = paths.i2(p);
        const int K = ADJ ? k + tn.x : k - tn.x;   // source column of element 0 (unwrapped)
        const bool lo0 = K < 0, hi0 = K >= M, lo1 = K + 1 < 0, hi1 = K + 1 >= M;
        const int s0 = lo0 ? K + M : (hi0 ? K - M : K);
        const bool split = s0 == M - 1;
        C c0, c1;
        if constexpr (F32) {
          unpack2(buf_ld4b(rtab, ADJ ? 8u * (uint32_t)s0 : 8u * (uint32_t)k, (uint32_t)p * M8),
                  c0, c1);
          if (ADJ && __builtin_amdgcn_ballot_w64(split) != 0) {
            const float2 cfx = __builtin_bit_cast(
                float2, __builtin_amdgcn_raw_buffer_load_b64(rtab, 0u, (uint32_t)p * M8, 0));
            if (split) c1 = cfx;
          }
        } else {   // one 16-byte entry per column
          const uint32_t k1 = ADJ ? (split ? 0u : (uint32_t)s0 + 1u) : (uint32_t)k + 1u;
          c0 = A::tab(rtab, TS * 8u * (ADJ ? (uint32_t)s0 : (uint32_t)k), TS * (uint32_t)p * M8);
          c1 = A::tab(rtab, TS * 8u * k1, TS * (uint32_t)p * M8);
        }
        if (ADJ) {
          c0 = A::conj(c0);
          c1 = A::conj(c1);
        }
        const int lc = full_cols ? s0 : K - col0;   // window column of element 0
        const int sh = ADJ ? tn.y : -tn.y;
        C e0[kLdsRows], e1[kLdsRows];
        window_reads(e0, e1, [&](int i) { return win + wrow(i, sh) * WC + lc; });
        if constexpr (WRAP) {
          // wrapped elements take W^n; selected per lane without a branch, so the
          // accumulators are not copied between two arms on every path
          C cw0 = c0, cw1 = c1;
          if (!ADJ) {
            const C wn = A::tab_s(wt, tn.y < 0 ? tn.y + N : tn.y);
            cw0 = A::mul(c0, cplx<C>(wn.x, hi0 ? -wn.y : wn.y));
            cw1 = A::mul(c1, cplx<C>(wn.x, hi1 ? -wn.y : wn.y));
          }
#pragma unroll
          for (int i = 0; i < kLdsRows; ++i) {
            const C w0 = cplx<C>(wl[i].x, hi0 ? wl[i].y : -wl[i].y);
            const C w1 = cplx<C>(wl[i].x, hi1 ? wl[i].y : -wl[i].y);
            A::mac(acc0[i], (lo0 || hi0) ? A::mul(cw0, w0) : c0, e0[i]);
            A::mac(acc1[i], (lo1 || hi1) ? A::mul(cw1, w1) : c1, e1[i]);
          }
        } else {
#pragma unroll
          for (int i = 0; i < kLdsRows; ++i) {
            A::mac(acc0[i], c0, e0[i]);
            A::mac(acc1[i], c1, e1[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < kLdsRows; ++i)
        if (j0 + i < nrows) sink((uint32_t)(l[i] * M + k), acc0[i], acc1[i], pf[i]);
    }
    };
    if (!strip_wraps && !full_rows)
      chunks(std::false_type{}, std::integral_constant<int, 0>{});
    else
      chunks(std::true_type{}, std::integral_constant<int, 2>{});
  }
  __syncthreads();   // the window region is free for the caller
}

// band_apply with nothing to prefetch: sink(q, v)
struct NoPref {
  __device__ __forceinline__ NoPre operator()(uint32_t) const { return NoPre{}; }
};
template <int R, int U, bool ADJ, int SD, class Src, class Sink>
__device__ __forceinline__ void band_apply(const FrameDev& F, int lb, int le, const Src& src,
                                           Sink sink) {
  band_apply<R, U, ADJ, SD>(F, lb, le, src, NoPref{},
                                [&](int q, float2 v, NoPre) { sink(q, v); });
}

// ---------------------------------------------------------------------------------------
// LDS-staged band application (frames with F.skc > 0, coefficients synthesised).
//
// The band is processed in blocks of ssb rows x skc delay columns (skc <= 256: one column
// per thread, kStageRows rows per thread).  For a block the workgroup first copies into
// LDS every source element its outputs can reach -- rows shifted by [nu_lo, nu_hi] and
// columns shifted by [tau_lo, tau_hi], both ranges widened to contain 0 so that the
// outputs' own elements are in the window too (whole rows when the column window would
// cover them, all N rows when the row window wraps the frame).  The copy goes straight from
// memory to LDS (buffer_load_dword ... lds): every load of the window is in flight at once
// and none occupies a VGPR.  Each staged vector (Src::kNV of them: c and the old p in
// phase A) has its own window; every path's gather then reads LDS.  Loads the outputs need
// besides the window (Out::pre) are issued before the copy is waited for.
// ---------------------------------------------------------------------------------------
template <bool ADJ, class Src, class Out>
__device__ __forceinline__ void staged_apply(const FrameDev& F, int lb, int le, float2* lds_gen,
                                             const Src& src, const Out& out) {
  constexpr int NV = Src::kNV;
  const int M = F.M, N = F.N, P = F.P;
  const int KC = F.skc, SB = F.ssb;
  const int tlo = F.tau_lo, thi = F.tau_hi, vlo = F.nu_lo, vhi = F.nu_hi;
  const int dtau = thi - tlo, dnu = vhi - vlo;
  const bool full_cols = KC + dtau >= M;
  const int TYc = kBlock / KC;
  const int tx = threadIdx.x % KC, ty = threadIdx.x / KC;
  const bool active = ty < TYc;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const KPairs paths = kpairs(F.paths);
  const KPairs wtab_s = kpairs(F.wtab);
  const GPairs rtab = gpairs(F.rtab);
  const GPairs wtab = gpairs(F.wtab);
  LdsC win[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) win[j] = lds_c(lds_gen) + j * F.swin;
  for (int sb0 = lb; sb0 < le; sb0 += SB) {
    const int sbn = min(SB, le - sb0);
    const bool full_rows = sbn + dnu >= N;
    const int WR = full_rows ? N : sbn + dnu;
    const int row0 = full_rows ? 0 : (ADJ ? sb0 + vlo : sb0 - vhi);
    // the thread's output rows in this block (rows past the block repeat its last row)
    int lrow[kStageRows];
    float2 wl[kStageRows];
#pragma unroll
    for (int i = 0; i < kStageRows; ++i) {
      lrow[i] = min(ty + i * TYc, sbn - 1);
      wl[i] = wtab.f(sb0 + lrow[i]);
    }
    for (int k0 = 0; k0 < M; k0 += KC) {
      const int kcn = min(KC, M - k0);
      const int WC = full_cols ? M : kcn + dtau;
      const int col0 = full_cols ? 0 : (ADJ ? k0 + tlo : k0 - thi);
      const int WS = (WC + 31) & ~31;        // LDS row stride: 32 elements per wave copy
      const int k = k0 + min(tx, kcn - 1);
      typename Out::Pre pre[kStageRows];
#pragma unroll
      for (int i = 0; i < kStageRows; ++i) pre[i] = out.pre((uint32_t)((sb0 + lrow[i]) * M + k));
      __syncthreads();                         // the previous block's readers are done
      // one wave copies 32 consecutive window elements of one row (two dwords per element)
      const int half = lane & 1;
      const int nch = WS >> 5;
      for (int r = wave; r < WR; r += kWaves) {
        int sr = row0 + r;
        sr += sr < 0 ? N : 0;
        sr -= sr >= N ? N : 0;
        const int rowoff = sr * M;
        for (int ch = 0; ch < nch; ++ch) {
          const int c = ch * 32 + (lane >> 1);
          if (c < WC) {
            int sc = col0 + c;
            sc += sc < 0 ? M : 0;
            sc -= sc >= M ? M : 0;
            const uint32_t voff = (uint32_t)(rowoff + sc) * 8u + (uint32_t)half * 4u;
#pragma unroll
            for (int j = 0; j < NV; ++j)
              __builtin_amdgcn_raw_ptr_buffer_load_lds(
                  src.rsrc(j), (lptr<void>)(win[j].p + r * WS + ch * 32), 4, voff, 0, 0, 0);
          }
        }
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (!active || tx >= kcn) continue;
      const int cc = tx;
      float2 acc[kStageRows];
#pragma unroll
      for (int i = 0; i < kStageRows; ++i) acc[i] = make_float2(0.f, 0.f);
      for (int p = 0; p < P; ++p) {
        const int2 tn = paths.i2(p);
        const int K = ADJ ? k + tn.x : k - tn.x;
        const int n = K < 0 ? -1 : (K >= M ? 1 : 0);
        const int kk = K - n * M;
        const float2 rv = rtab.f(p * M + (ADJ ? kk : k));
        const float2 cf = ADJ ? make_float2(rv.x, -rv.y) : rv;
        float2 cw = cf;
        if (!ADJ) {
          const float2 wn = wtab_s.f(tn.y < 0 ? tn.y + N : tn.y);
          cw = cmulf(cf, make_float2(wn.x, n > 0 ? -wn.y : wn.y));
        }
        const int lc = full_cols ? kk : (ADJ ? cc + (tn.x - tlo) : cc + (thi - tn.x));
#pragma unroll
        for (int i = 0; i < kStageRows; ++i) {
          const int rr = lrow[i];
          int lr;
          if (full_rows) {
            lr = ADJ ? sb0 + rr + tn.y : sb0 + rr - tn.y;
            lr += lr < 0 ? N : 0;
            lr -= lr >= N ? N : 0;
          } else {
            lr = ADJ ? rr + (tn.y - vlo) : rr + (vhi - tn.y);
          }
          const int at = lr * WS + lc;
          float2 v[NV];
#pragma unroll
          for (int j = 0; j < NV; ++j) v[j] = win[j].ld(at);
          const float2 w = make_float2(wl[i].x, n > 0 ? wl[i].y : -wl[i].y);
          const float2 cr = cmulf(cw, w);
          cmacf(acc[i], n != 0 ? cr : cf, src.combine(v));
        }
      }
      // own elements (shift 0) are in the window
      const int oc = full_cols ? k : cc + (ADJ ? -tlo : thi);
#pragma unroll
      for (int i = 0; i < kStageRows; ++i) {
        const int rr = ty + i * TYc;
        if (rr < sbn) {
          const int orow = full_rows ? sb0 + rr : rr + (ADJ ? -vlo : vhi);
          float2 own[NV];
#pragma unroll
          for (int j = 0; j < NV; ++j) own[j] = win[j].ld(orow * WS + oc);
          out.put((uint32_t)((sb0 + rr) * M + k), acc[i], pre[i], own);
        }
      }
    }
  }
}

// Band application of H / H^H.  GM says where the gathers read from: memory (kGmDirect),
// LDS windows of the staged geometry (kGmStaged: frames with F.skc > 0), or the windowed
// paired gathers (kGmLds: frames with F.lpk > 0, else memory).  out.pre(q) issues the
// loads output q needs besides the source; out.put(q, v, pre, own) receives it with own[] =
// the source vectors' elements at q.
constexpr int kGmDirect = 0, kGmStaged = 1, kGmLds = 2;

template <bool ADJ, int SD, int GM, int R = kRows, int UP = kPaths, class Src, class Out>
__device__ __forceinline__ void apply_band(const FrameDev& F, int lb, int le, float2* lds,
                                           const Src& src, const Out& out) {
  if constexpr (GM == kGmStaged && SD == kDNone && Src::kStageable) {
    staged_apply<ADJ>(F, lb, le, lds, src, out);
    return;
  }
  if constexpr (GM == kGmLds && SD == kDNone) {
    if constexpr (std::is_same<Src, SrcBuf>::value) {
      if (pairs_ok(F) && lds_window_fits(F, lb, le)) {   // same bits as the direct pairs
        static_assert(!Out::kOwn, "the windowed pairs pass no own elements");
        lds_apply_pairs<ADJ, ArithF32>(
            F, lb, le, src, lds, [&](uint32_t u) { return out.pre2(u); },
            [&](uint32_t q, float2 v0, float2 v1, const typename Out::Pre2& pr) {
              out.put2(q, v0, v1, pr, nullptr, nullptr);
            });
        return;
      }
    }
    // otherwise (not pairs-aligned, a window that does not fit, or a source the window
    // does not take): gathered straight from memory one element per lane (this kind keeps
    // the registers of the paired gathers for the window's form)
    struct PreOwnL {
      typename Out::Pre pre;
      float2 own[Src::kNV];
    };
    band_apply<R, UP, ADJ, SD>(
        F, lb, le, src,
        [&](uint32_t u) {
          PreOwnL po;
          po.pre = out.pre(u);
          if (Out::kOwn) src.own(u, po.own);
          return po;
        },
        [&](int q, float2 v, const PreOwnL& po) { out.put((uint32_t)q, v, po.pre, po.own); });
    return;
  }
  if constexpr (SD == kDNone && Src::kPairs) {
    if (pairs_ok(F)) {
      struct PreOwn2 {
        typename Out::Pre2 pre;
        float2 own0[Src::kNV], own1[Src::kNV];
      };
      band_apply_pairs<R, (UP < kPairPaths ? UP : kPairPaths), ADJ>(
          F, lb, le, src,
          [&](uint32_t u) {
            PreOwn2 po;
            po.pre = out.pre2(u);
            if (Out::kOwn) src.own2(u, po.own0, po.own1);
            return po;
          },
          [&](uint32_t q, float2 v0, float2 v1, const PreOwn2& po) {
            out.put2(q, v0, v1, po.pre, po.own0, po.own1);
          });
      return;
    }
  }
  struct PreOwn {
    typename Out::Pre pre;
    float2 own[Src::kNV];
  };
  band_apply<R, UP, ADJ, SD>(
      F, lb, le, src,
      [&](uint32_t u) {
        PreOwn po;
        po.pre = out.pre(u);
        if (Out::kOwn) src.own(u, po.own);
        return po;
      },
      [&](int q, float2 v, const PreOwn& po) { out.put((uint32_t)q, v, po.pre, po.own); });
}

// ---------------------------------------------------------------------------------------
// Windowed band application of H (ADJ = false) or H^H (ADJ = true) over a strip.
//
// The workgroup owns delay columns [k0, k0 + W) of one frame over all N Doppler rows.
// Output row l of path p reads source row l + s_l(p) at column k + s_k(p) (H: s = (-tau,
// -nu); H^H: s = (+tau, +nu)).  The rows are produced RC at a time.  The source rows that a
// chunk reaches -- rows [l0 + s_l,min, l0 + RC - 1 + s_l,max], columns [k0 + s_k,min,
// k0 + W - 1 + s_k,max] (both ranges widened to contain 0) -- sit in an LDS ring of
// NB = 2 RC + d_nu rows: while a chunk is computed from LDS, the RC rows the next chunk adds
// are read from memory into registers (every read of the chunk issued together, none under
// a branch), then written to their ring slots, which no workgroup-mate still reads (the ring
// holds two chunks of new rows besides the shared ones), and one barrier per chunk
// publishes them.  Each source element is read from memory once per strip (plus the
// d_nu-row head of the ring and the d_tau-column margin shared with the neighbour strips),
// instead of once per path.
//
// Thread (tx, ty) keeps column k = k0 + tx: the P coefficients R_p[k] (H) or conj R_p[<k +
// tau_p>_M] (H^H) and the delay-wrap flags of that column stay in registers for the whole
// strip.  Coefficients, wrap factors and the order of the sum over paths are exactly those
// of band_apply, so the two give identical bits.
//
// src: a source view (SrcBuf, SrcDir, SrcBf16): load(i) reads element i of the frame,
// value(raw) forms it.  pref(q) issues the loads output q needs besides the source;
// sink(q, v, pre) receives output q.  W is a multiple of 64 dividing kBlock, P <= kWinPaths,
// RC * ceil((W + d_tau) / 64) <= kWaves * kWinLoads (the host guarantees all three).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int mod_floor(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

template <bool ADJ, int RPT, class Src, class Pref, class Sink>
__device__ __forceinline__ void win_apply(const FrameDev& F, int k0, float2* lds_gen,
                                          const Src& src, Pref pref, Sink sink) {
  const int M = F.M, N = F.N, P = F.P;
  const int W = F.win_w, RC = F.win_rc;
  const int TY = kBlock / W;
  const int tx = (int)threadIdx.x % W;
  const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.x / W);
  const int smin_k = ADJ ? F.tau_lo : -F.tau_hi, smax_k = ADJ ? F.tau_hi : -F.tau_lo;
  const int smin_l = ADJ ? F.nu_lo : -F.nu_hi, smax_l = ADJ ? F.nu_hi : -F.nu_lo;
  const int WC = W + (smax_k - smin_k);
  const int NB = 2 * RC + (smax_l - smin_l);
  const int cbase = k0 + smin_k;                // unwrapped column of window column 0
  const int k = k0 + tx;
  const KPairs paths = kpairs(F.paths);
  const KPairs wtab_s = kpairs(F.wtab);
  const GPairs rtab = gpairs(F.rtab);
  const LdsC ring = lds_c(lds_gen);

  // per-path shifts (wave-uniform, loaded once: scalar loads inside the gather loop would
  // make every wait for them also wait for the ring reads in flight), and per-path column
  // state: coefficient and delay-wrap flags (lo: bit p, hi: bit 16 + p)
  int2 tns[kWinPaths];
#pragma unroll
  for (int p = 0; p < kWinPaths; ++p) tns[p] = p < P ? paths.i2(p) : make_int2(0, 0);
  float2 cf[kWinPaths];
  uint32_t wrap = 0u;
#pragma unroll
  for (int p = 0; p < kWinPaths; ++p) {
    if (p < P) {
      const int2 tn = tns[p];
      const int K = ADJ ? k + tn.x : k - tn.x;
      const bool lo = K < 0, hi = K >= M;
      const int kk = lo ? K + M : (hi ? K - M : K);
      const float2 r = rtab.f((int64_t)p * M + (ADJ ? kk : k));
      cf[p] = ADJ ? make_float2(r.x, -r.y) : r;
      wrap |= (lo ? 1u : 0u) << p;
      wrap |= (hi ? 1u : 0u) << (16 + p);
    } else {
      cf[p] = make_float2(0.f, 0.f);
    }
  }

  // staging map: a chunk's RC rows x WC window columns are cut into pieces of 64
  // consecutive columns of one row; wave w takes pieces w, w + kWaves, ... (at most
  // kWinLoads), so a piece's row is wave-uniform and each lane reads one element (lanes
  // past the end of a row re-read its last element and store nothing)
  const int NBLK = (WC + 63) / 64;
  const int pieces = RC * NBLK;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = (int)threadIdx.x & 63;
  typename Src::Raw buf[kWinLoads];
  // read the RC source rows starting at unwrapped row r0 into registers / write them to
  // the ring slots of ring positions rp0 ..
  auto issue = [&](int r0) {
    const int rw0 = mod_floor(r0, N);
#pragma unroll
    for (int m = 0; m < kWinLoads; ++m) {
      const int pc = wave + m * kWaves;
      if (pc < pieces) {
        const int i = pc / NBLK, b = pc - i * NBLK;
        int r = rw0 + i;
        r -= r >= N ? N : 0;
        int col = cbase + min(b * 64 + lane, WC - 1);
        col += col < 0 ? M : 0;
        col -= col >= M ? M : 0;
        buf[m] = src.load((uint32_t)r * (uint32_t)M + (uint32_t)col);
      }
    }
  };
  auto commit = [&](int rp0) {
    const int s0 = rp0 % NB;
#pragma unroll
    for (int m = 0; m < kWinLoads; ++m) {
      const int pc = wave + m * kWaves;
      if (pc < pieces) {
        const int i = pc / NBLK, b = pc - i * NBLK;
        const int c = b * 64 + lane;
        int sl = s0 + i;
        sl -= sl >= NB ? NB : 0;
        if (c < WC) ring.st(sl * WC + c, src.value(buf[m]));
      }
    }
  };

  // the head of the ring: rows smin_l .. RC - 1 + smax_l (d_nu + RC rows, RC at a time)
  const int head = RC + (smax_l - smin_l);
  for (int h = 0; h < head; h += RC) {
    issue(smin_l + h);
    commit(h);
  }
  __syncthreads();

  const int nch = (N + RC - 1) / RC;
  for (int j = 0; j < nch; ++j) {
    const int l0 = j * RC;
    // the next chunk's new rows, in flight during this chunk's arithmetic
    const bool more = j + 1 < nch;
    if (more) issue(l0 + RC + smax_l);
    int l[RPT];
    float2 acc[RPT];
    decltype(pref(0u)) pf[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      l[i] = min(l0 + ty + i * TY, N - 1);
      acc[i] = make_float2(0.f, 0.f);
      pf[i] = pref((uint32_t)(l[i] * M + k));
    }
    const int jb = l0 % NB;                       // ring slot of unwrapped row l0 + smin_l
#pragma unroll
    for (int p = 0; p < kWinPaths; ++p) {
      if (p < P) {
        const int2 tn = tns[p];
        const int sk = ADJ ? tn.x : -tn.x, sl = ADJ ? tn.y : -tn.y;
        const uint32_t col = (uint32_t)(tx + sk - smin_k);
        const bool lo = (wrap >> p) & 1u, hi = (wrap >> (16 + p)) & 1u;
        float2 v[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          // ring position of source row l + sl, relative to row l0 + smin_l
          int sp = jb + (l[i] - l0) + (sl - smin_l);
          sp -= sp >= NB ? NB : 0;
          v[i] = ring.ld(sp * WC + (int)col);
        }
        if (__builtin_amdgcn_ballot_w64(lo || hi) != 0) {
          float2 cw = cf[p];
          if (!ADJ) {
            const float2 wn = wtab_s.f(tn.y < 0 ? tn.y + N : tn.y);
            cw = cmulf(cf[p], make_float2(wn.x, hi ? -wn.y : wn.y));
          }
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const float2 wli = wtab_s.f(l[i]);     // only waves holding a delay wrap
            const float2 w = make_float2(wli.x, hi ? wli.y : -wli.y);
            const float2 c = (lo || hi) ? cmulf(cw, w) : cf[p];
            cmacf(acc[i], c, v[i]);
          }
        } else {
#pragma unroll
          for (int i = 0; i < RPT; ++i) cmacf(acc[i], cf[p], v[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (l0 + ty + i * TY < N) sink(l[i] * M + k, acc[i], pf[i]);
    if (more) commit(l0 + head);
    __syncthreads();
  }
}

// win_apply for the frame's rows per thread and chunk (2 or 4; the host guarantees one).
template <bool ADJ, class Src, class Pref, class Sink>
__device__ __forceinline__ void win_apply_any(const FrameDev& F, int k0, float2* lds,
                                              const Src& src, Pref pref, Sink sink) {
#ifdef OTFS_WIN_RPT_ONLY
  win_apply<ADJ, OTFS_WIN_RPT_ONLY>(F, k0, lds, src, pref, sink);
#else
  if (F.win_rc / (kBlock / F.win_w) == 4)
    win_apply<ADJ, 4>(F, k0, lds, src, pref, sink);
  else
    win_apply<ADJ, 2>(F, k0, lds, src, pref, sink);
#endif
}

// ---------------------------------------------------------------------------------------
// hard decisions (Eq. demod): nearest square-QAM level per axis, ties to the upper level
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int decide_axis(float v, float s, int m) {
  float t = __fmul_rn(v, s);
  t = __fadd_rn(t, (float)m);
  t = __fmul_rn(t, 0.5f);
  t = t == t ? t : 0.f;                         // NaN -> lowest level
  t = fminf(fmaxf(t, 0.f), (float)(m - 1));
  return (int)floorf(t);
}
__device__ __forceinline__ uint8_t decide(float2 x, float s, int m) {
  return (uint8_t)(decide_axis(x.x, s, m) * m + decide_axis(x.y, s, m));
}

struct FrameVecs {
  const void* y;
  float2* x;
  uint8_t* sym;
  otfs_frame_stats* stats;
  bool ybf16;
};
__device__ __forceinline__ FrameVecs frame_vecs(const FrameDev& F, const Bases& B) {
  FrameVecs v;
  v.ybf16 = (F.flags & OTFS_Y_BF16) != 0;
  if (B.y)
    v.y = static_cast<const char*>(B.y) + F.off * (v.ybf16 ? 4 : 8);
  else
    v.y = F.y;
  v.x = B.x ? B.x + F.off : F.x;
  v.sym = B.sym ? B.sym + F.off : F.sym;
  v.stats = B.stats ? B.stats + F.index : F.stats;
  return v;
}

// Final x update (if pending), decisions and statistics of one tile.
__device__ __forceinline__ void finish_tile(const FrameDev& F, const WorkItem& wi, const FrameVecs& V,
                            const FrameState& s, const float2* pcur, bool xpending,
                            int status) {
  const int M = F.M;
  const bool dec = V.sym != nullptr && F.qside > 0;
  auto one = [&](int64_t q) {
    float2 xv = V.x[q];
    if (xpending) {
      xv = axpyf(s.alpha, pcur[q], xv);
      V.x[q] = xv;
    }
    if (dec) V.sym[q] = decide(xv, F.qscale, F.qside);
  };
  const int cols = wi.k_end - wi.k_begin;
  if (cols == M) {   // a band of whole rows: one contiguous range
    const int64_t q0 = (int64_t)wi.l_begin * M, q1 = (int64_t)wi.l_end * M;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock) one(q);
  } else {           // a strip: cols divides kBlock, so each thread keeps one column
    const int tx = (int)threadIdx.x % cols, ty = (int)threadIdx.x / cols;
    for (int l = wi.l_begin + ty; l < wi.l_end; l += kBlock / cols)
      one((int64_t)l * M + wi.k_begin + tx);
  }
  if (wi.tile == 0 && threadIdx.x == 0) {
    if (V.stats) {
      otfs_frame_stats st;
      st.iters = s.iter;
      st.rel_res = s.rel;
      st.status = status;
      st.tiles = F.T;
      *V.stats = st;
    }
    FrameState o = s;
    o.status = status;
    o.pending = 0;
    *F.st = o;
  }
}

// ---------------------------------------------------------------------------------------
// One workgroup's share of one frame's CG loop inside the fused persistent kernel.
//
// Schedule per iteration xi (three per-frame barriers, each vector pass reads/writes the
// band once):
//   A: p_new = c + beta p_old and x += alpha p_old for the band (the direction and x
//      updates of iteration xi-1, deferred), t = H p_new with the gathered p_new values
//      recomputed from c and p_old exactly as their owners compute them;     | barrier
//   B: a = H^H t + lam p_new, partial Re(p_new^H a);                         | barrier
//   C: alpha = c_norm / Re(p^H a); c -= alpha a, partial ||c||^2;            | barrier
//   then every workgroup forms the same c_norm' in the same order, tests the stop rule
//   and sets beta = c_norm' / c_norm.  x += alpha p stays pending until the next A (or
//   the finish).
// FP64 true-residual refresh: after every k-th iteration (refresh_every) the C pass also
// applies x += alpha p, and the frame leaves the launch with its state marked `refresh`.
// The refresh launches (k_refresh_u, k_refresh_c) then replace c by the true residual
// H^H (y - H x) - lam x formed in FP64 and leave its FP64 partial norms; the next fused
// launch resumes the frame with the stop test on that norm.
// ---------------------------------------------------------------------------------------
struct LaunchCtx {
  unsigned* abort_flag;
  uint64_t timeout;
  int xcd_local;     // barrier coherence mode (see frame_barrier)
};

// FP64 true-residual refresh of one tile through the LDS window of the windowed paired
// gathers (used by the refresh launches and, inside the fused launch, by the windowed kind).
// The residual is formed in FP64 (no cancellation between y and Hx) and kept in FP32.
__device__ __forceinline__ float2 refresh_res(float2 yv, double2 v) {
  return make_float2((float)((double)yv.x - v.x), (float)((double)yv.y - v.y));
}
// u = y - H x over the band (FP64 tables and sums)
__device__ __forceinline__ void refresh_u_window(const FrameDev& F, const WorkItem& wi,
                                                 const FrameVecs& V, float2* lds) {
  const int64_t E = (int64_t)F.M * F.N;
  const CVec u = cvec(F.u, E);
  const SrcBuf xs{buf_rsrc(V.x, E * 8)};
  struct Y2 {
    float2 a, b;
  };
  lds_apply_pairs<false, ArithF64>(
      F, wi.l_begin, wi.l_end, xs, lds,
      [&](uint32_t q) { return Y2{load_y(V.y, q, V.ybf16), load_y(V.y, q + 1u, V.ybf16)}; },
      [&](uint32_t q, double2 v0, double2 v1, const Y2& yv) {
        u.st2(q, refresh_res(yv.a, v0), refresh_res(yv.b, v1));
      });
}
// c = H^H u - lam x over the band, rounded to FP32; returns this thread's FP64 partial of
// ||c||^2
__device__ __forceinline__ double refresh_c_window(const FrameDev& F, const WorkItem& wi,
                                                   const FrameVecs& V, float2* lds) {
  const int64_t E = (int64_t)F.M * F.N;
  const double lam = (double)F.lam;
  const CVec cv = cvec(F.c, E), xv = cvec(V.x, E);
  const SrcBuf us{buf_rsrc(F.u, E * 8)};
  double acc = 0.0;
  auto cval = [&](double2 v, float2 x) {
    return make_float2((float)(v.x - lam * (double)x.x), (float)(v.y - lam * (double)x.y));
  };
  auto nrm = [&](float2 cf) {
    acc = fma((double)cf.x, (double)cf.x, acc);
    acc = fma((double)cf.y, (double)cf.y, acc);
  };
  struct X2 {
    float2 a, b;
  };
  lds_apply_pairs<true, ArithF64>(
      F, wi.l_begin, wi.l_end, us, lds,
      [&](uint32_t q) {
        X2 r;
        xv.ld2(q, r.a, r.b);
        return r;
      },
      [&](uint32_t q, double2 v0, double2 v1, const X2& x) {
        const float2 c0 = cval(v0, x.a), c1 = cval(v1, x.b);
        cv.st2(q, c0, c1);
        nrm(c0);
        nrm(c1);
      });
  return acc;
}
// Whether every tile of the frame refreshes through its window (a decision the same for all
// tiles of the frame: its bands are floor(N / T) or ceil(N / T) rows)
__device__ __forceinline__ bool frame_windows_fit(const FrameDev& F) {
  return F.lpk > 0 && pairs_ok(F) && lds_window_fits(F, 0, F.N / F.T) &&
         lds_window_fits(F, 0, (F.N + F.T - 1) / F.T);
}

// A frame's state as every lane holds it: read through the vector path (other workgroups
// write it), then taken from the first lane, so that what is derived from it (which
// direction buffer is current, and the buffer descriptors built on that) stays in scalar
// registers instead of every buffer access being repeated per distinct descriptor.
__device__ __forceinline__ FrameState uniform_state(const FrameState* p) {
  FrameState s = *p;
  s.iter = __builtin_amdgcn_readfirstlane(s.iter);
  s.status = __builtin_amdgcn_readfirstlane(s.status);
  s.pbuf = __builtin_amdgcn_readfirstlane(s.pbuf);
  s.pending = __builtin_amdgcn_readfirstlane(s.pending);
  s.init = __builtin_amdgcn_readfirstlane(s.init);
  s.refresh = __builtin_amdgcn_readfirstlane(s.refresh);
  return s;
}

// GM: where the gathers read from (kGmDirect, kGmStaged, kGmLds).  FDIR: the H pass forms
// p' = c + beta p inside its gathers (direct-fd kind).
template <int SD, int GM, bool FDIR = false>
__device__ __forceinline__ void cg_item(const FrameDev& F, const WorkItem& wi, int budget, const Bases& B,
                        const LaunchCtx& L, float* red, int* sflag, float2* lds) {
  // the stored-table reads leave fewer registers for gathers in flight
  constexpr int RR = SD != kDNone ? 2 : kRows;
  // elements per thread in flight in the element-wise passes (the windowed kind has the
  // registers for more)
  constexpr int ECK = GM == kGmLds ? kElemChunkLds : kElemChunk;
  const FrameVecs V = frame_vecs(F, B);
  FrameState s = uniform_state(F.st);
  if (s.status != OTFS_FRAME_RUNNING) return;
  const int M = F.M, T = F.T;
  const int lb = wi.l_begin, le = wi.l_end;
  const int64_t q0 = (int64_t)lb * M, q1 = (int64_t)le * M;
  const float lam = F.lam;
  const int64_t E = (int64_t)M * F.N;
  const uint32_t u0 = (uint32_t)q0, u1 = (uint32_t)q1;
  const CVec cv = cvec(F.c, E), tv = cvec(F.t, E), av = cvec(F.a, E), xv = cvec(V.x, E);
  unsigned nbar = 0;
  auto bar = [&]() -> bool {
    if (T == 1) {
      __syncthreads();
      return true;
    }
    nbar += (unsigned)T;
    return frame_barrier(F.bar, nbar, L.xcd_local != 0, L.abort_flag, L.timeout, sflag);
  };
  // tiles whose rows the H pass (rows l - nu) and the H^H pass (rows l + nu) read
  const int span = le - lb + (F.nu_hi - F.nu_lo);
  const TileRange rd_h = tiles_of_rows(lb - F.nu_hi, span, F.N, T);
  const TileRange rd_hh = tiles_of_rows(lb + F.nu_lo, span, F.N, T);
  unsigned npub = 0;
  auto halo = [&](const TileRange& tr) -> bool {
    if (T == 1) {
      __syncthreads();
      return true;
    }
    tile_publish(F.prog + wi.tile, L.xcd_local != 0);
    ++npub;
    return halo_wait(F.prog, T, tr, npub, L.xcd_local != 0, L.abort_flag, L.timeout, sflag);
  };
  auto fail_timeout = [&]() {
    if (wi.tile == 0 && threadIdx.x == 0) {
      FrameState o = s;
      o.status = OTFS_FRAME_TIMEOUT;
      *F.st = o;
      if (V.stats) {
        otfs_frame_stats st{s.iter, s.rel, OTFS_FRAME_TIMEOUT, T};
        *V.stats = st;
      }
    }
  };

  // ---- b = H^H y; x = 0; c = p = b; c_norm_0 = ||b||^2 (the initialisation of Algorithm 1) ----
  if (!s.init) {
    float acc = 0.f;
    const OutInit out{cv, cvec(F.p0, E), xv, &acc};
    if (V.ybf16)
      apply_band<true, SD, GM, RR>(F, lb, le, lds, SrcBf16{buf_rsrc(V.y, E * 4)}, out);
    else
      apply_band<true, SD, GM, RR>(F, lb, le, lds, SrcBuf{buf_rsrc(V.y, E * 8)}, out);
    const float bs = block_sum(acc, red);
    if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
    if (!bar()) return fail_timeout();
    const float cn0 = tile_sum(F.part_cc, T);
    s.init = 1;
    s.iter = 0;
    s.pbuf = 0;
    s.pending = 0;
    s.cn = cn0;
    s.cn0 = cn0;
    s.alpha = 0.f;
    s.beta = 0.f;
    s.rel = cn0 > 0.f ? 1.f : 0.f;
    if (!(cn0 > 0.f)) {
      const int st = cn0 == 0.f ? OTFS_FRAME_CONVERGED : OTFS_FRAME_NONFINITE;
      return finish_tile(F, wi, V, s, F.p0, false, st);
    }
  }

  // After the C pass of iteration s.iter: the stop test on the residual norm cn_new, then
  // beta for the next direction.  xpend: x += alpha p of that iteration is still to do.
  // Returns false when the frame is finished (its tile already finalised).
  auto next = [&](float cn_new, bool xpend, float2* pcur) -> bool {
    s.rel = sqrtf(cn_new / s.cn0);
    int st = OTFS_FRAME_RUNNING;
    if (!isfinite(cn_new))
      st = OTFS_FRAME_NONFINITE;
    else if (F.tol > 0.f && s.rel <= F.tol)
      st = OTFS_FRAME_CONVERGED;
    else if (s.iter >= F.max_iters)
      st = OTFS_FRAME_CAPPED;
    if (st != OTFS_FRAME_RUNNING) {
      finish_tile(F, wi, V, s, pcur, xpend, st);
      return false;
    }
    s.beta = cn_new / s.cn;
    s.cn = cn_new;
    s.pending = (xpend ? 1 : 0) | 2;
    return true;
  };
  if (s.refresh) {   // resume after the refresh launches: the true residual's norm
    s.refresh = 0;
    if (!next((float)tile_sum_d(F.part_d, T), false, F.p0)) return;
  }

  for (int step = 0; step < budget; ++step) {
    const int xi = s.iter + 1;
    float2* const pold_g = s.pbuf ? F.p1 : F.p0;
    float2* const pnew_g = s.pbuf ? F.p0 : F.p1;
    const CVec pov = cvec(pold_g, E), pnv = cvec(pnew_g, E);
    // the refresh launches follow this iteration: x += alpha p is applied in the C pass
    const bool refresh_due =
        F.refresh_every > 0 && xi % F.refresh_every == 0 && xi < F.max_iters;
    // iteration 1 has no pending update: beta = 0 gives p_new = c = b exactly
    const bool xp = (s.pending & 1) != 0;
    const float al = s.alpha, be = (s.pending & 2) ? s.beta : 0.f;

    // ---- A: deferred updates of the band, t = H p ----
    if constexpr (GM == kGmStaged) {
      // c and the old p are staged together; p' = c + beta p is formed from the windows
      apply_band<false, SD, kGmStaged, RR>(F, lb, le, lds, SrcDir{cv.r, pov.r, be},
                                           OutA{tv, pnv, xv, al, be, xp});
    } else if constexpr (FDIR) {
      // p' = c + beta p_old formed from both vectors at every gather (two loads each: fewer
      // paths in flight), stored once for the own rows with x += alpha p_old
      apply_band<false, SD, kGmDirect, kFdRows, kFdPaths>(F, lb, le, lds,
                                                         SrcDir{cv.r, pov.r, be},
                                                         OutA{tv, pnv, xv, al, be, xp});
    } else {
      // A1: p' = c + beta p_old and x += alpha p_old over the band, stored once
      if (pairs_ok(F)) {   // two elements per lane and access (16-byte loads and stores)
        constexpr int EP = ECK / 2;
        for (uint32_t u = u0 + 2u * threadIdx.x; u < u1; u += 2u * kBlock * EP) {
          float2 c0[EP], c1[EP], p0[EP], p1[EP], x0[EP], x1[EP];
#pragma unroll
          for (int j = 0; j < EP; ++j) {
            const uint32_t w = min(u + (uint32_t)(2 * j * kBlock), u1 - 2u);
            cv.ld2<kNtElem>(w, c0[j], c1[j]);
            pov.ld2<kNtElem>(w, p0[j], p1[j]);
            if (xp) xv.ld2<kNtElem>(w, x0[j], x1[j]);
          }
#pragma unroll
          for (int j = 0; j < EP; ++j) {
            const uint32_t w = u + (uint32_t)(2 * j * kBlock);
            if (w < u1) {
              pnv.st2<kNtP>(w, axpyf(be, p0[j], c0[j]), axpyf(be, p1[j], c1[j]));
              if (xp) xv.st2<kNtElemSt>(w, axpyf(al, p0[j], x0[j]), axpyf(al, p1[j], x1[j]));
            }
          }
        }
      } else
      for (uint32_t u = u0 + threadIdx.x; u < u1; u += kBlock * ECK) {
        float2 c[ECK], po[ECK], xo[ECK];
#pragma unroll
        for (int j = 0; j < ECK; ++j) {
          const uint32_t w = min(u + (uint32_t)(j * kBlock), u1 - 1u);
          c[j] = cv.ld<kNtElem>(w);
          po[j] = pov.ld<kNtElem>(w);
          if (xp) xo[j] = xv.ld<kNtElem>(w);
        }
#pragma unroll
        for (int j = 0; j < ECK; ++j) {
          const uint32_t w = u + (uint32_t)(j * kBlock);
          if (w < u1) {
            pnv.st<kNtP>(w, axpyf(be, po[j], c[j]));
            if (xp) xv.st<kNtElemSt>(w, axpyf(al, po[j], xo[j]));
          }
        }
      }
      if (!halo(rd_h)) return fail_timeout();
      // A2: t = H p' (one load per gather, or through LDS windows)
      if (kNtT && F.stream_t)
        apply_band<false, SD, GM, RR>(F, lb, le, lds, SrcBuf{pnv.r}, OutStore<true>{tv});
      else
        apply_band<false, SD, GM, RR>(F, lb, le, lds, SrcBuf{pnv.r}, OutStore<false>{tv});
    }
    if (!halo(rd_hh)) return fail_timeout();

    // ---- B: a = H^H t + lam p, partial Re(p^H a) ----
    {
      float acc = 0.f;
      apply_band<true, SD, GM, RR>(F, lb, le, lds, SrcBuf{tv.r}, OutB{av, pnv, lam, &acc});
      const float bs = block_sum(acc, red);
      if (threadIdx.x == 0) F.part_pa[wi.tile] = bs;
    }
    if (!bar()) return fail_timeout();
    s.pbuf ^= 1;
    s.pending = 0;                                   // both deferred updates are applied

    const float den = tile_sum(F.part_pa, T);
    const float alpha = s.cn / den;
    if (!(den > 0.f) || !isfinite(alpha)) {          // x already holds x_{xi-1}
      const int st = (isfinite(den) && isfinite(s.cn)) ? OTFS_FRAME_BREAKDOWN
                                                        : OTFS_FRAME_NONFINITE;
      return finish_tile(F, wi, V, s, pnew_g, false, st);
    }

    // ---- C: c -= alpha a, partial ||c||^2 ----
    {
      float acc = 0.f;
      // EC elements per thread at a time, all loads issued first (past the band's end the
      // last element is re-read and nothing is stored)
      constexpr int EC = FDIR ? kElemChunkFd : ECK;
      if (pairs_ok(F)) {   // two elements per lane and access; the same sums per element
        constexpr int EP = EC / 2;
        for (uint32_t u = u0 + 2u * threadIdx.x; u < u1; u += 2u * kBlock * EP) {
          float2 a0[EP], a1[EP], c0[EP], c1[EP];
#pragma unroll
          for (int j = 0; j < EP; ++j) {
            const uint32_t w = min(u + (uint32_t)(2 * j * kBlock), u1 - 2u);
            av.ld2<kNtElem>(w, a0[j], a1[j]);
            cv.ld2<kNtElem>(w, c0[j], c1[j]);
          }
#pragma unroll
          for (int j = 0; j < EP; ++j) {
            const uint32_t w = u + (uint32_t)(2 * j * kBlock);
            if (w < u1) {
              const float2 n0 = axpyf(-alpha, a0[j], c0[j]), n1 = axpyf(-alpha, a1[j], c1[j]);
              cv.st2<kNtElemSt>(w, n0, n1);
              acc = fmaf(n0.x, n0.x, acc);
              acc = fmaf(n0.y, n0.y, acc);
              acc = fmaf(n1.x, n1.x, acc);
              acc = fmaf(n1.y, n1.y, acc);
            }
          }
        }
      } else
      for (uint32_t u = u0 + threadIdx.x; u < u1; u += kBlock * EC) {
        float2 a[EC], c[EC];
#pragma unroll
        for (int j = 0; j < EC; ++j) {
          const uint32_t w = min(u + (uint32_t)(j * kBlock), u1 - 1u);
          a[j] = av.ld<kNtElem>(w);
          c[j] = cv.ld<kNtElem>(w);
        }
#pragma unroll
        for (int j = 0; j < EC; ++j) {
          const uint32_t w = u + (uint32_t)(j * kBlock);
          if (w < u1) {
            const float2 cn = axpyf(-alpha, a[j], c[j]);
            cv.st<kNtElemSt>(w, cn);
            acc = fmaf(cn.x, cn.x, acc);
            acc = fmaf(cn.y, cn.y, acc);
          }
        }
      }
      if (refresh_due) {   // x += alpha p' before the refresh launches read x
        if (pairs_ok(F)) {   // as in the passes above: EP pairs per thread in flight
          constexpr int EP = ECK / 2;
          for (uint32_t u = u0 + 2u * threadIdx.x; u < u1; u += 2u * kBlock * EP) {
            float2 p0[EP], p1[EP], x0[EP], x1[EP];
#pragma unroll
            for (int j = 0; j < EP; ++j) {
              const uint32_t w = min(u + (uint32_t)(2 * j * kBlock), u1 - 2u);
              pnv.ld2(w, p0[j], p1[j]);
              xv.ld2(w, x0[j], x1[j]);
            }
#pragma unroll
            for (int j = 0; j < EP; ++j) {
              const uint32_t w = u + (uint32_t)(2 * j * kBlock);
              if (w < u1) xv.st2(w, axpyf(alpha, p0[j], x0[j]), axpyf(alpha, p1[j], x1[j]));
            }
          }
        } else {
          for (uint32_t u = u0 + threadIdx.x; u < u1; u += kBlock)
            xv.st(u, axpyf(alpha, pnv.ld(u), xv.ld(u)));
        }
      }
      const float bs = block_sum(acc, red);
      if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
    }
    if (!bar()) return fail_timeout();
    const float cn_new = tile_sum(F.part_cc, T);
    s.iter = xi;
    s.alpha = alpha;
    if (refresh_due) {
      if (!isfinite(cn_new)) return finish_tile(F, wi, V, s, pnew_g, false, OTFS_FRAME_NONFINITE);
      if constexpr (GM == kGmLds) {
        if (frame_windows_fit(F)) {
          // The true residual inside this launch, by the same steps as the refresh launches:
          // u = y - H x (x is final in every tile after the barrier above), the
          // neighbouring tiles' u, then c = H^H u - lam x with its FP64 norm.
          refresh_u_window(F, wi, V, lds);
          if (!halo(rd_hh)) return fail_timeout();
          const double bs = block_sum_d(refresh_c_window(F, wi, V, lds),
                                        reinterpret_cast<double*>(red));
          if (threadIdx.x == 0) F.part_d[wi.tile] = bs;
          if (!bar()) return fail_timeout();
          s.pending = 0;
          if (!next((float)tile_sum_d(F.part_d, T), false, F.p0)) return;
          continue;
        }
      }
      // leave the launch: the refresh launches form the true residual of x
      s.refresh = 1;
      s.pending = 0;
      if (wi.tile == 0 && threadIdx.x == 0) *F.st = s;
      return;
    }
    if (!next(cn_new, true, pnew_g)) return;
  }
  // iteration budget of this launch used up: keep the state for the next launch
  if (wi.tile == 0 && threadIdx.x == 0) *F.st = s;
}

// ---------------------------------------------------------------------------------------
// One strip's share of one frame's CG loop with windowed gathers (frames with win_w > 0).
//
// The schedule and the arithmetic are those of the direct kind with the direction formed
// inside the H pass (cg_item<.., FDIR = true>); only the tile shape and where the gathers
// read from change.  A tile is a strip of W delay columns over all N Doppler rows, so the
// Doppler wrap is inside the tile and only the delay range crosses tiles.  Per iteration:
//   A: t = H p', p' = c + beta p_old formed as each source row enters the LDS ring; the own
//      elements store p' and x += alpha p_old (the deferred updates); no wait before it,
//      since c and p_old were last written before the previous frame barrier;
//   wait for the strips whose columns the H^H window covers;
//   B: a = H^H t + lam p', partial Re(p'^H a);                               | barrier
//   C: c -= alpha a, partial ||c||^2 over the strip;                         | barrier
// ---------------------------------------------------------------------------------------
struct OwnCPX {      // own elements the H pass needs besides the window
  float2 c, p, x;
};

__device__ void cg_item_win(const FrameDev& F, const WorkItem& wi, int budget, const Bases& B,
                            const LaunchCtx& L, float* red, int* sflag, float2* lds) {
  const FrameVecs V = frame_vecs(F, B);
  FrameState s = uniform_state(F.st);
  if (s.status != OTFS_FRAME_RUNNING) return;
  const int M = F.M, N = F.N, T = F.T, W = F.win_w;
  const int k0 = wi.k_begin;
  const int TY = kBlock / W;
  const int tx = (int)threadIdx.x % W;
  const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.x / W);
  const float lam = F.lam;
  const int64_t E = (int64_t)M * N;
  const CVec cv = cvec(F.c, E), tv = cvec(F.t, E), av = cvec(F.a, E), xv = cvec(V.x, E);
  unsigned nbar = 0;
  auto bar = [&]() -> bool {
    if (T == 1) {
      __syncthreads();
      return true;
    }
    nbar += (unsigned)T;
    return frame_barrier(F.bar, nbar, L.xcd_local != 0, L.abort_flag, L.timeout, sflag);
  };
  // strips whose columns the H^H pass gathers: [k0 + tau_lo, k0 + W - 1 + tau_hi] (mod M)
  const TileRange rd_hh = tiles_of_rows(k0 + F.tau_lo, W + (F.tau_hi - F.tau_lo), M, T);
  unsigned npub = 0;
  auto halo = [&](const TileRange& tr) -> bool {
    if (T == 1) {
      __syncthreads();
      return true;
    }
    tile_publish(F.prog + wi.tile, L.xcd_local != 0);
    ++npub;
    return halo_wait(F.prog, T, tr, npub, L.xcd_local != 0, L.abort_flag, L.timeout, sflag);
  };
  auto fail_timeout = [&]() {
    if (wi.tile == 0 && threadIdx.x == 0) {
      FrameState o = s;
      o.status = OTFS_FRAME_TIMEOUT;
      *F.st = o;
      if (V.stats) {
        otfs_frame_stats st{s.iter, s.rel, OTFS_FRAME_TIMEOUT, T};
        *V.stats = st;
      }
    }
  };

  // ---- b = H^H y; x = 0; c = p = b; c_norm_0 = ||b||^2 ----
  if (!s.init) {
    float acc = 0.f;
    const CVec p0v = cvec(F.p0, E);
    auto sink = [&](int q, float2 v, NoPre) {
      cv.st((uint32_t)q, v);
      p0v.st((uint32_t)q, v);
      xv.st((uint32_t)q, make_float2(0.f, 0.f));
      acc = fmaf(v.x, v.x, acc);
      acc = fmaf(v.y, v.y, acc);
    };
    if (V.ybf16)
      win_apply_any<true>(F, k0, lds, SrcBf16{buf_rsrc(V.y, E * 4)}, NoPref{}, sink);
    else
      win_apply_any<true>(F, k0, lds, SrcBuf{buf_rsrc(V.y, E * 8)}, NoPref{}, sink);
    const float bs = block_sum(acc, red);
    if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
    if (!bar()) return fail_timeout();
    const float cn0 = tile_sum(F.part_cc, T);
    s.init = 1;
    s.iter = 0;
    s.pbuf = 0;
    s.pending = 0;
    s.cn = cn0;
    s.cn0 = cn0;
    s.alpha = 0.f;
    s.beta = 0.f;
    s.rel = cn0 > 0.f ? 1.f : 0.f;
    if (!(cn0 > 0.f)) {
      const int st = cn0 == 0.f ? OTFS_FRAME_CONVERGED : OTFS_FRAME_NONFINITE;
      return finish_tile(F, wi, V, s, F.p0, false, st);
    }
  }

  for (int step = 0; step < budget; ++step) {
    const int xi = s.iter + 1;
    float2* const pold_g = s.pbuf ? F.p1 : F.p0;
    float2* const pnew_g = s.pbuf ? F.p0 : F.p1;
    const CVec pov = cvec(pold_g, E), pnv = cvec(pnew_g, E);
    const bool xp = (s.pending & 1) != 0;
    const float al = s.alpha, be = (s.pending & 2) ? s.beta : 0.f;

    // ---- A: t = H p' with p' = c + beta p_old formed in the ring; own p', x updates ----
    win_apply_any<false>(
        F, k0, lds, SrcDir{cv.r, pov.r, be},
        [&](uint32_t q) {
          OwnCPX o;
          o.c = cv.ld(q);
          o.p = pov.ld(q);
          o.x = xp ? xv.ld(q) : make_float2(0.f, 0.f);
          return o;
        },
        [&](int q, float2 v, const OwnCPX& o) {
          tv.st((uint32_t)q, v);
          pnv.st((uint32_t)q, axpyf(be, o.p, o.c));
          if (xp) xv.st((uint32_t)q, axpyf(al, o.p, o.x));
        });
    if (!halo(rd_hh)) return fail_timeout();

    // ---- B: a = H^H t + lam p', partial Re(p'^H a) ----
    {
      float acc = 0.f;
      win_apply_any<true>(
          F, k0, lds, SrcBuf{tv.r}, [&](uint32_t q) { return pnv.ld(q); },
          [&](int q, float2 v, const float2& p) {
            const float2 a = axpyf(lam, p, v);
            av.st<kNtB>((uint32_t)q, a);
            acc = fmaf(p.x, a.x, acc);
            acc = fmaf(p.y, a.y, acc);
          });
      const float bs = block_sum(acc, red);
      if (threadIdx.x == 0) F.part_pa[wi.tile] = bs;
    }
    if (!bar()) return fail_timeout();
    s.pbuf ^= 1;
    s.pending = 0;
    const float den = tile_sum(F.part_pa, T);
    const float alpha = s.cn / den;
    if (!(den > 0.f) || !isfinite(alpha)) {
      const int st = (isfinite(den) && isfinite(s.cn)) ? OTFS_FRAME_BREAKDOWN
                                                        : OTFS_FRAME_NONFINITE;
      return finish_tile(F, wi, V, s, pnew_g, false, st);
    }

    // ---- C: c -= alpha a over the strip, partial ||c||^2 ----
    {
      float acc = 0.f;
      constexpr int EC = kElemChunkFd;
      for (int r = ty; r < N; r += TY * EC) {
        float2 a[EC], c[EC];
#pragma unroll
        for (int j = 0; j < EC; ++j) {
          const uint32_t w = (uint32_t)(min(r + j * TY, N - 1) * M + k0 + tx);
          a[j] = av.ld<kNtElem>(w);
          c[j] = cv.ld<kNtElem>(w);
        }
#pragma unroll
        for (int j = 0; j < EC; ++j) {
          if (r + j * TY < N) {
            const uint32_t w = (uint32_t)((r + j * TY) * M + k0 + tx);
            const float2 cn = axpyf(-alpha, a[j], c[j]);
            cv.st<kNtElemSt>(w, cn);
            acc = fmaf(cn.x, cn.x, acc);
            acc = fmaf(cn.y, cn.y, acc);
          }
        }
      }
      const float bs = block_sum(acc, red);
      if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
    }
    if (!bar()) return fail_timeout();
    const float cn_new = tile_sum(F.part_cc, T);
    s.iter = xi;
    s.alpha = alpha;
    s.rel = sqrtf(cn_new / s.cn0);
    if (!isfinite(cn_new)) return finish_tile(F, wi, V, s, pnew_g, true, OTFS_FRAME_NONFINITE);
    if (F.tol > 0.f && s.rel <= F.tol)
      return finish_tile(F, wi, V, s, pnew_g, true, OTFS_FRAME_CONVERGED);
    if (xi >= F.max_iters) return finish_tile(F, wi, V, s, pnew_g, true, OTFS_FRAME_CAPPED);
    s.beta = cn_new / s.cn;
    s.cn = cn_new;
    s.pending = 3;
  }
  if (wi.tile == 0 && threadIdx.x == 0) *F.st = s;
}

// ---------------------------------------------------------------------------------------
// A small frame handled by one workgroup with x, c, p, t and a resident in LDS for the
// whole solve: y is read once (b = H^H y), x_hat and the decisions are written once, and
// every pass in between runs out of LDS with no per-frame barrier.  Same schedule and
// arithmetic as cg_item for one tile (the deferred updates are applied in place before
// the gathers, all of which are then of the finished p').  When a serving step ends
// before the frame does, x, c and p are saved to the frame's vectors (p in p0) and
// reloaded by the next launch.
// ---------------------------------------------------------------------------------------
__device__ void cg_item_resident(const FrameDev& F, int budget, const Bases& B, float* red,
                                 float2* lds) {
  const FrameVecs V = frame_vecs(F, B);
  FrameState s = uniform_state(F.st);
  if (s.status != OTFS_FRAME_RUNNING) return;
  const int N = F.N;
  const int E = F.M * F.N;
  const LdsC xs = lds_c(lds);
  const LdsC cs = xs + E;
  const LdsC ps = xs + 2 * E;
  const LdsC ts = xs + 3 * E;
  const LdsC as = xs + 4 * E;
  const float lam = F.lam;
  const bool dec = V.sym != nullptr && F.qside > 0;
  auto finish = [&](bool xpending, int status) {
    for (int q = threadIdx.x; q < E; q += kBlock) {
      float2 xv = xs.ld(q);
      if (xpending) xv = axpyf(s.alpha, ps.ld(q), xv);
      V.x[q] = xv;
      if (dec) V.sym[q] = decide(xv, F.qscale, F.qside);
    }
    if (threadIdx.x == 0) {
      if (V.stats) {
        otfs_frame_stats st{s.iter, s.rel, status, 1};
        *V.stats = st;
      }
      FrameState o = s;
      o.status = status;
      o.pending = 0;
      *F.st = o;
    }
  };

  if (!s.init) {
    // b = H^H y; x = 0; c = p = b; c_norm_0 = ||b||^2 (the initialisation of Algorithm 1)
    float acc = 0.f;
    auto sink = [&](int q, float2 v) {
      cs.st(q, v);
      ps.st(q, v);
      xs.st(q, make_float2(0.f, 0.f));
      acc = fmaf(v.x, v.x, acc);
      acc = fmaf(v.y, v.y, acc);
    };
    if (V.ybf16)
      band_apply<kResRows, kResPaths, true, false>(F, 0, N, SrcBf16{buf_rsrc(V.y, (int64_t)E * 4)}, sink);
    else
      band_apply<kResRows, kResPaths, true, false>(F, 0, N, SrcBuf{buf_rsrc(V.y, (int64_t)E * 8)}, sink);
    const float cn0 = block_sum(acc, red);
    s.init = 1;
    s.iter = 0;
    s.pbuf = 0;
    s.pending = 0;
    s.cn = cn0;
    s.cn0 = cn0;
    s.alpha = 0.f;
    s.beta = 0.f;
    s.rel = cn0 > 0.f ? 1.f : 0.f;
    if (!(cn0 > 0.f)) return finish(false, cn0 == 0.f ? OTFS_FRAME_CONVERGED : OTFS_FRAME_NONFINITE);
  } else {
    for (int q = threadIdx.x; q < E; q += kBlock) {
      xs.st(q, V.x[q]);
      cs.st(q, F.c[q]);
      ps.st(q, F.p0[q]);
    }
    __syncthreads();
  }

  for (int step = 0; step < budget; ++step) {
    const int xi = s.iter + 1;
    const bool xp = (s.pending & 1) != 0;
    const float al = s.alpha, be = (s.pending & 2) ? s.beta : 0.f;
    // A: deferred updates in place, then t = H p'
    for (int q = threadIdx.x; q < E; q += kBlock) {
      const float2 po = ps.ld(q);
      if (xp) xs.st(q, axpyf(al, po, xs.ld(q)));
      ps.st(q, axpyf(be, po, cs.ld(q)));
    }
    __syncthreads();
    band_apply<kResRows, kResPaths, false, false>(
        F, 0, N, SrcLds{ps}, [&](int q, float2 v) { ts.st(q, v); });
    __syncthreads();
    // B: a = H^H t + lam p', Re(p'^H a)
    float acc = 0.f;
    band_apply<kResRows, kResPaths, true, false>(
        F, 0, N, SrcLds{ts},
        [&](int q, float2 v) {
          const float2 p = ps.ld(q);
          const float2 a = axpyf(lam, p, v);
          as.st(q, a);
          acc = fmaf(p.x, a.x, acc);
          acc = fmaf(p.y, a.y, acc);
        });
    const float den = block_sum(acc, red);
    s.pending = 0;
    const float alpha = s.cn / den;
    if (!(den > 0.f) || !isfinite(alpha)) {
      const int st = (isfinite(den) && isfinite(s.cn)) ? OTFS_FRAME_BREAKDOWN
                                                        : OTFS_FRAME_NONFINITE;
      return finish(false, st);
    }
    // C: c -= alpha a, ||c||^2
    acc = 0.f;
#pragma unroll 4
    for (int q = threadIdx.x; q < E; q += kBlock) {
      const float2 c = axpyf(-alpha, as.ld(q), cs.ld(q));
      cs.st(q, c);
      acc = fmaf(c.x, c.x, acc);
      acc = fmaf(c.y, c.y, acc);
    }
    const float cn_new = block_sum(acc, red);
    s.iter = xi;
    s.alpha = alpha;
    s.rel = sqrtf(cn_new / s.cn0);
    if (!isfinite(cn_new)) return finish(true, OTFS_FRAME_NONFINITE);
    if (F.tol > 0.f && s.rel <= F.tol) return finish(true, OTFS_FRAME_CONVERGED);
    if (xi >= F.max_iters) return finish(true, OTFS_FRAME_CAPPED);
    s.beta = cn_new / s.cn;
    s.cn = cn_new;
    s.pending = 3;
  }
  // iteration budget of this launch used up: save the vectors and the state
  for (int q = threadIdx.x; q < E; q += kBlock) {
    V.x[q] = xs.ld(q);
    F.c[q] = cs.ld(q);
    F.p0[q] = ps.ld(q);
  }
  if (threadIdx.x == 0) {
    s.pbuf = 0;
    *F.st = s;
  }
}

// XCC (XCD) this wave runs on, from the hardware register XCC_ID, bits [3:0].
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg((15 << 11) | (0 << 6) | 20) & 0xfu);
}

// Work queues: group g owns items qitems[qrange[g].x .. qrange[g].y); its workgroups take
// them in order with an atomic cursor.  In XCD-local mode a workgroup serves the group of
// the XCD it runs on, so every frame (all of whose tiles sit in one group) is handled by
// workgroups sharing one L2.  A frame's tiles are consecutive in its group's queue and a
// group never has fewer resident workgroups than a frame has tiles, so the first frame
// with an untaken tile is always being completed: the per-frame barriers cannot deadlock.
#ifndef OTFS_WIN_MIN_WAVES
#define OTFS_WIN_MIN_WAVES 2
#endif
// Waves per SIMD the compiler must leave room for: the direct kinds take the whole
// register file of a CU for one 512-thread workgroup (256 VGPRs per lane: the paired
// gathers keep 16 reads of 16 bytes in flight per lane), the LDS kinds keep two per CU.
#ifndef OTFS_LDS_MIN_WAVES
#define OTFS_LDS_MIN_WAVES 4
#endif
constexpr int fused_min_waves(int kind) {
  return kind == kKindWindowed ? OTFS_WIN_MIN_WAVES
                               : ((kind == kKindDirect || kind == kKindDirectFD || kind == kKindLds)
                                      ? OTFS_FUSED_MIN_WAVES
                                      : OTFS_LDS_MIN_WAVES);
}
template <int SD, int KIND>
__global__ __launch_bounds__(kBlock, fused_min_waves(KIND)) void k_cg_fused(const FrameDev* __restrict__ frames,
                                                     const WorkItem* __restrict__ items,
                                                     const int32_t* __restrict__ qitems,
                                                     const int2* __restrict__ qrange,
                                                     unsigned* __restrict__ qhead, int ngroups,
                                                     int budget, Bases B, LaunchCtx L) {
  __shared__ double red_d[kWaves];   // FP32 sums use its first kWaves floats
  float* const red = reinterpret_cast<float*>(red_d);
  __shared__ int sflag;
  __shared__ int s_item;
  extern __shared__ float2 stage_lds[];
  // Data this launch reads may have been written by other kernels, copies or XCDs since
  // this XCD's L2 last saw it, and the per-frame barriers of XCD-local mode never
  // invalidate the L2: take one device-wide acquire before the first read, and publish
  // this workgroup's results device-wide before it exits.
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const int g = L.xcd_local ? xcc_id() : 0;
  if (g >= ngroups) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    return;
  }
  const int2 r = qrange[g];
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned j = __hip_atomic_fetch_add(&qhead[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_item = (int)j < r.y - r.x ? qitems[r.x + (int)j] : -1;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: descriptors in SGPRs
    __syncthreads();
    if (it < 0) break;
    const WorkItem wi = items[it];
    const FrameDev& F = frames[wi.frame];
    if constexpr (KIND == kKindResident)
      cg_item_resident(F, budget, B, red, stage_lds);
    else if constexpr (KIND == kKindWindowed)
      cg_item_win(F, wi, budget, B, L, red, &sflag, stage_lds);
    else
      cg_item<SD, KIND == kKindStaged ? kGmStaged : (KIND == kKindLds ? kGmLds : kGmDirect),
              KIND == kKindDirectFD>(F, wi, budget, B, L, red, &sflag,
                                                              stage_lds);
    __syncthreads();
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

__global__ void k_xcc_probe(int* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

// ---------------------------------------------------------------------------------------
// FP64 true-residual refresh of the frames whose state is marked `refresh` (they left the
// fused launch after the C pass of every k-th iteration, with x already updated).  One
// workgroup per tile; no cross-tile synchronisation inside a launch: the two launches are
// ordered by the stream.
//   k_refresh_u: u = y - H x, formed in FP64 from the FP32 x (FP64 tables, FP64 sums);
//   k_refresh_c: c = H^H u - lam x, rounded to FP32, and the FP64 partial of ||c||^2.
// k_refresh_u also clears the frame's barrier and neighbour counters for the next fused
// launch of the same solve.
// ---------------------------------------------------------------------------------------
#ifndef OTFS_REF_ROWS
#define OTFS_REF_ROWS 8
#endif
#ifndef OTFS_REF_MIN_WAVES
#define OTFS_REF_MIN_WAVES 2
#endif
// rows per thread chunk in the FP64 gathers: each path's FP64 coefficient (16 bytes per
// column) is read once per chunk, so tall chunks keep the table reads small next to the
// gathered data; one workgroup per CU leaves the registers for them
constexpr int kRefRows = OTFS_REF_ROWS;
constexpr int kRefPaths = 4;   // paths in flight together
// The refresh of a tile reads its gathers through the LDS window of the windowed paired
// gathers when the frame has that geometry, the window fits the launch's LDS and the
// frame's vectors split into 16-byte pairs.
// Item of this workgroup in the refresh launches.  Workgroup b runs on XCD b % nxcd; the
// workgroups of one XCD take consecutive items (the items of a frame are consecutive), so
// the tiles of a frame, whose windows share the rows of the Doppler range, read them
// through one L2.  A bijection of [0, nitems) for any nitems and nxcd >= 1.
__device__ __forceinline__ int refresh_item(int nitems, int nxcd) {
  if (nxcd <= 1) return (int)blockIdx.x;
  const int b = (int)blockIdx.x, x = b % nxcd;
  int o = 0;
  for (int y = 0; y < x; ++y) o += (nitems - y + nxcd - 1) / nxcd;
  return o + b / nxcd;
}
__device__ __forceinline__ bool ref_lds_ok(const FrameDev& F, const WorkItem& wi, int lds_bytes) {
  return F.lpk > 0 && pairs_ok(F) && F.lwr * F.lwc * (int)sizeof(float2) <= lds_bytes &&
         lds_window_fits(F, wi.l_begin, wi.l_end);
}

__global__ __launch_bounds__(kBlock, OTFS_REF_MIN_WAVES) void k_refresh_u(const FrameDev* __restrict__ frames,
                                                      const WorkItem* __restrict__ items, Bases B,
                                                      unsigned* qhead, int nq, int lds_bytes,
                                                      int nxcd) {
  extern __shared__ float2 ref_lds[];
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const WorkItem wi = items[refresh_item((int)gridDim.x, nxcd)];
  const FrameDev& F = frames[wi.frame];
  if (blockIdx.x == 0 && (int)threadIdx.x < nq) qhead[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    F.prog[wi.tile] = 0u;
    if (wi.tile == 0) *F.bar = 0u;
  }
  if (F.st->refresh == 0 || F.st->status != OTFS_FRAME_RUNNING) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    return;
  }
  const FrameVecs V = frame_vecs(F, B);
  if (ref_lds_ok(F, wi, lds_bytes)) {
    refresh_u_window(F, wi, V, ref_lds);
  } else {
    const int64_t E = (int64_t)F.M * F.N;
    const CVec u = cvec(F.u, E);
    const SrcBuf xs{buf_rsrc(V.x, E * 8)};
    band_apply<kRefRows, kRefPaths, false, kDNone>(
        F, wi.l_begin, wi.l_end, xs, [&](uint32_t q) { return load_y(V.y, q, V.ybf16); },
        [&](int q, double2 v, float2 yv) { u.st((uint32_t)q, refresh_res(yv, v)); }, ArithF64{});
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

__global__ __launch_bounds__(kBlock, OTFS_REF_MIN_WAVES) void k_refresh_c(const FrameDev* __restrict__ frames,
                                                      const WorkItem* __restrict__ items, Bases B,
                                                      int lds_bytes, int nxcd) {
  __shared__ double redd[kWaves];
  extern __shared__ float2 ref_lds[];
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const WorkItem wi = items[refresh_item((int)gridDim.x, nxcd)];
  const FrameDev& F = frames[wi.frame];
  if (F.st->refresh == 0 || F.st->status != OTFS_FRAME_RUNNING) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    return;
  }
  const FrameVecs V = frame_vecs(F, B);
  double acc = 0.0;
  if (ref_lds_ok(F, wi, lds_bytes)) {
    acc = refresh_c_window(F, wi, V, ref_lds);
  } else {
    const int64_t E = (int64_t)F.M * F.N;
    const double lam = (double)F.lam;
    const CVec cv = cvec(F.c, E), xv = cvec(V.x, E);
    const SrcBuf us{buf_rsrc(F.u, E * 8)};
    auto cval = [&](double2 v, float2 x) {
      return make_float2((float)(v.x - lam * (double)x.x), (float)(v.y - lam * (double)x.y));
    };
    auto nrm = [&](float2 cf) {
      acc = fma((double)cf.x, (double)cf.x, acc);
      acc = fma((double)cf.y, (double)cf.y, acc);
    };
    band_apply<kRefRows, kRefPaths, true, kDNone>(
        F, wi.l_begin, wi.l_end, us, [&](uint32_t q) { return xv.ld(q); },
        [&](int q, double2 v, float2 x) {
          const float2 cf = cval(v, x);
          cv.st((uint32_t)q, cf);
          nrm(cf);
        },
        ArithF64{});
  }
  const double bs = block_sum_d(acc, redd);
  if (threadIdx.x == 0) F.part_d[wi.tile] = bs;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// ---------------------------------------------------------------------------------------
// standalone operator applications (one workgroup per tile)
// ---------------------------------------------------------------------------------------
template <bool ADJ, int SD>
__global__ __launch_bounds__(kBlock) void k_apply(const FrameDev* __restrict__ frames,
                                                  const WorkItem* __restrict__ items,
                                                  const float2* __restrict__ in,
                                                  float2* __restrict__ out) {
  const WorkItem wi = items[blockIdx.x];
  const FrameDev& F = frames[wi.frame];
  extern __shared__ float2 stage_lds[];
  const int64_t E = (int64_t)F.M * F.N;
  const CVec dst = cvec(out + F.off, E);
  if (SD == kDNone && F.win_w > 0)
    win_apply_any<ADJ>(F, wi.k_begin, stage_lds, src_vec(in + F.off, E), NoPref{},
                       [&](int q, float2 v, NoPre) { dst.st((uint32_t)q, v); });
  else if (SD == kDNone && F.skc > 0)
    apply_band<ADJ, SD, kGmStaged>(F, wi.l_begin, wi.l_end, stage_lds, src_vec(in + F.off, E),
                                   OutStore<>{dst});
  else
    apply_band<ADJ, SD, kGmDirect>(F, wi.l_begin, wi.l_end, stage_lds, src_vec(in + F.off, E),
                                   OutStore<>{dst});
}

__global__ void k_reset(const FrameDev* __restrict__ frames, int nframes, unsigned* abort_flag,
                        unsigned* qhead, int ngroups) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0 && abort_flag) *abort_flag = 0u;
  if (qhead && t < ngroups) qhead[t] = 0u;
  for (int i = t; i < nframes; i += gridDim.x * blockDim.x) {
    const FrameDev& F = frames[i];
    *F.bar = 0u;
    for (int j = 0; j < F.T; ++j) F.prog[j] = 0u;
    FrameState s;
    s.iter = 0;
    s.status = OTFS_FRAME_RUNNING;
    s.pbuf = 0;
    s.pending = 0;
    s.cn = s.cn0 = s.alpha = s.beta = s.rel = 0.f;
    s.init = 0;
    s.cn_hist[0] = s.cn_hist[1] = 0.f;
    s.refresh = 0;
    *F.st = s;
  }
}

// Between two serving steps: clear the barrier counters, queue cursors and abort word,
// and mark each frame's stats slot as running; the CG state of the frames is kept.
__global__ void k_step_reset(const FrameDev* __restrict__ frames, int nframes,
                             unsigned* abort_flag, unsigned* qhead, int ngroups) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0 && abort_flag) *abort_flag = 0u;
  if (qhead && t < ngroups) qhead[t] = 0u;
  for (int i = t; i < nframes; i += gridDim.x * blockDim.x) {
    const FrameDev& F = frames[i];
    *F.bar = 0u;
    for (int j = 0; j < F.T; ++j) F.prog[j] = 0u;
    if (F.stats) {
      otfs_frame_stats st{0, 0.f, OTFS_FRAME_RUNNING, F.T};
      *F.stats = st;
    }
  }
}

// Stored coefficients D_{p,q} (Eq. D_definition) of every frame, as bf16 pairs (SD =
// kDBf16, rounded to nearest even) or complex64 (kDC64): the FP32 value the on-the-fly
// synthesis forms for a gather of row q, path p.
template <int SD>
__global__ __launch_bounds__(kBlock) void k_build_d(const FrameDev* __restrict__ frames,
                                                    const WorkItem* __restrict__ items) {
  const WorkItem wi = items[blockIdx.x];
  const FrameDev& F = frames[wi.frame];
  const int M = F.M, N = F.N;
  const int64_t E = (int64_t)M * N;
  for (int64_t q = (int64_t)wi.l_begin * M + threadIdx.x; q < (int64_t)wi.l_end * M;
       q += kBlock) {
    const int k = (int)(q % M), l = (int)(q / M);
    for (int p = 0; p < F.P; ++p) {
      const int2 tn = F.paths[p];
      const int K = k - tn.x;
      const int n = K < 0 ? -1 : (K >= M ? 1 : 0);
      int ls = l - tn.y;
      ls += ls < 0 ? N : 0;
      ls -= ls >= N ? N : 0;
      float2 c = F.rtab[p * M + k];
      if (n != 0) {
        float2 w = F.wtab[ls];
        if (n < 0) w.y = -w.y;
        c = cmulf(c, w);
      }
      if constexpr (SD == kDC64)
        static_cast<float2*>(const_cast<void*>(F.dtab))[p * E + q] = c;
      else
        static_cast<uint32_t*>(const_cast<void*>(F.dtab))[p * E + q] =
            f32_to_bf16(c.x) | (f32_to_bf16(c.y) << 16);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Bits of the hard decisions (Eq. demod demaps each decided symbol to its bits; the map is
// a reflected Gray code per axis, g = i XOR (i >> 1), in-phase bits above quadrature bits)
// and bit-error counts against the transmitted symbol indices.  One workgroup per work
// item; every frame's count is the sum of its tiles' integer partials (exact, any order).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t gray_sym(uint32_t idx, uint32_t m, uint32_t b) {
  const uint32_t iI = idx / m, iQ = idx - iI * m;
  return ((iI ^ (iI >> 1)) << b) | (iQ ^ (iQ >> 1));
}
__device__ __forceinline__ uint32_t log2u(uint32_t m) { return 31u - __builtin_clz(m); }

__device__ void tile_bit_errors(const FrameDev& F, const WorkItem& wi, const uint8_t* sym,
                                const uint8_t* tx, unsigned long long* err, int* red) {
  const uint32_t m = (uint32_t)F.qside, b = log2u(m);
  const int M = F.M;
  uint32_t cnt = 0;
  auto one = [&](int64_t q) { cnt += __popc(gray_sym(sym[q], m, b) ^ gray_sym(tx[q], m, b)); };
  const int cols = wi.k_end - wi.k_begin;
  if (cols == M) {
    for (int64_t q = (int64_t)wi.l_begin * M + threadIdx.x; q < (int64_t)wi.l_end * M; q += kBlock)
      one(q);
  } else {
    const int tx0 = (int)threadIdx.x % cols, ty = (int)threadIdx.x / cols;
    for (int l = wi.l_begin + ty; l < wi.l_end; l += kBlock / cols) one((int64_t)l * M + wi.k_begin + tx0);
  }
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (int)cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int i = 0; i < kWaves; ++i) tot += (unsigned)red[i];
    atomicAdd(err, tot);
  }
}

__global__ __launch_bounds__(kBlock) void k_bit_errors(const FrameDev* __restrict__ frames,
                                                       const WorkItem* __restrict__ items,
                                                       const uint8_t* sym, const uint8_t* tx,
                                                       unsigned long long* errs) {
  __shared__ int red[kWaves];
  const WorkItem wi = items[blockIdx.x];
  const FrameDev& F = frames[wi.frame];
  if (F.qside <= 0) return;
  tile_bit_errors(F, wi, sym + F.off, tx + F.off, errs + F.index, red);
}

// Bit errors of the estimates after the current iteration (CG trace): a frame still
// running holds x with its last update x += alpha p' pending, so its decisions are taken on
// x + alpha p'; a finished frame's x and decisions are final.  The decisions are written to
// the caller's buffer (sym), then counted against tx into errs[F.index].
__global__ __launch_bounds__(kBlock) void k_trace_errors(const FrameDev* __restrict__ frames,
                                                         const WorkItem* __restrict__ items,
                                                         Bases B, const uint8_t* tx,
                                                         unsigned long long* errs) {
  __shared__ int red[kWaves];
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const WorkItem wi = items[blockIdx.x];
  const FrameDev& F = frames[wi.frame];
  if (F.qside <= 0) return;
  const FrameVecs V = frame_vecs(F, B);
  const FrameState s = *F.st;
  const bool pend = s.status == OTFS_FRAME_RUNNING && (s.pending & 1) != 0;
  const float2* pcur = s.pbuf ? F.p1 : F.p0;
  const int M = F.M;
  for (int64_t q = (int64_t)wi.l_begin * M + threadIdx.x; q < (int64_t)wi.l_end * M; q += kBlock) {
    float2 xv = V.x[q];
    if (pend) xv = axpyf(s.alpha, pcur[q], xv);
    V.sym[q] = decide(xv, F.qscale, F.qside);
  }
  __syncthreads();
  tile_bit_errors(F, wi, V.sym, tx + F.off, errs + F.index, red);
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ---------------------------------------------------------------------------------------
// Structured-sparse channel from a received pilot frame (Sec. IV-A "Hadamard product" and
// Sec. IV-B "Dominant path determination"), one workgroup per frame.
//
// The pilot is one impulse at (K0, L0) = (M/2, N/2).  The estimate of the effective channel
// on the received grid is h[k, l] = Y[k, l] E_twist[k, l] with
// E_twist[k, l] = e^{-j 2 pi K0 (l - L0) / (MN)} (Eqs. heff_exp, heff_hadamard); bin (k, l)
// stands for the path with shifts (tau, nu) = (k - K0, l - L0).  The dominant paths are the
// bins with |h| > theta (Eq. heff_thres), tested as |h|^2 > theta^2 in FP32 on the
// estimate rounded to FP32.  The workgroup walks the frame in vector order, kBlock bins at
// a time, and compacts the selected bins in that order (wave ballots and a prefix over the
// waves); the first F.pcap become the frame's paths: the table of shifts, P, the shift
// ranges, and the delay-ramp tables R_p[k] = h_p e^{j 2 pi nu_p (k - tau_p) / (MN)} (FP32,
// and FP64 where the frame keeps them for the refresh), each phase from its integer
// numerator reduced modulo MN before one FP64 sine / cosine.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double2 unit_phasor(int64_t num, int64_t mn) {
  num %= mn;
  if (num < 0) num += mn;
  double sn, cs;
  sincospi(2.0 * ((double)num / (double)mn), &sn, &cs);
  return make_double2(cs, sn);
}

__global__ __launch_bounds__(kBlock) void k_pilot_paths(FrameDev* __restrict__ frames,
                                                        const float2* __restrict__ ypilot,
                                                        float theta, int32_t* npaths) {
  __shared__ int wcount[kWaves];
  __shared__ float2 s_gain[kMaxPathsDev];
  __shared__ int2 s_tn[kMaxPathsDev];
  FrameDev& F = frames[blockIdx.x];
  const int M = F.M, N = F.N, K0 = M / 2, L0 = N / 2;
  const int64_t E = (int64_t)M * N, MN = E;
  const int cap = min(F.pcap, kMaxPathsDev);
  const GPairs yp = gpairs(ypilot + F.off);
  const float th2 = __fmul_rn(theta, theta);
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  int base = 0;
  for (int64_t q0 = 0; q0 < E; q0 += kBlock) {
    const int64_t q = q0 + threadIdx.x;
    bool sel = false;
    float2 h = make_float2(0.f, 0.f);
    int k = 0, l = 0;
    if (q < E) {
      l = (int)(q / M);
      k = (int)(q - (int64_t)l * M);
      const double2 tw = unit_phasor(-(int64_t)K0 * (l - L0), MN);
      const float2 y = yp.f(q);
      h = make_float2((float)((double)y.x * tw.x - (double)y.y * tw.y),
                      (float)((double)y.x * tw.y + (double)y.y * tw.x));
      sel = __fadd_rn(__fmul_rn(h.x, h.x), __fmul_rn(h.y, h.y)) > th2;
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(sel);
    const int before = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (lane == 0) wcount[wave] = __popcll(m);
    __syncthreads();
    int woff = 0, total = 0;
    for (int w = 0; w < kWaves; ++w) {
      const int c = wcount[w];
      woff += w < wave ? c : 0;
      total += c;
    }
    const int idx = base + woff + before;
    if (sel && idx < cap) {
      s_tn[idx] = make_int2(k - K0, l - L0);
      s_gain[idx] = h;
    }
    base += total;
    __syncthreads();
  }
  const int P = base < cap ? base : cap;
  int2* const paths = const_cast<int2*>(F.paths);
  float2* const rtab = const_cast<float2*>(F.rtab);
  double2* const rtab64 = const_cast<double2*>(F.rtab64);
  if ((int)threadIdx.x < P) paths[threadIdx.x] = s_tn[threadIdx.x];
  for (int i = threadIdx.x; i < P * M; i += kBlock) {
    const int p = i / M, k = i - p * M;
    const int2 tn = s_tn[p];
    const double2 ph = unit_phasor((int64_t)tn.y * (k - tn.x), MN);
    const double hr = (double)s_gain[p].x, hi = (double)s_gain[p].y;
    const double2 r = make_double2(hr * ph.x - hi * ph.y, hr * ph.y + hi * ph.x);
    rtab[i] = make_float2((float)r.x, (float)r.y);
    if (rtab64) rtab64[i] = r;
  }
  if (threadIdx.x == 0) {
    // shift ranges, widened to contain 0 as the host forms them
    int tlo = 0, thi = 0, vlo = 0, vhi = 0;
    for (int p = 0; p < P; ++p) {
      tlo = min(tlo, s_tn[p].x);
      thi = max(thi, s_tn[p].x);
      vlo = min(vlo, s_tn[p].y);
      vhi = max(vhi, s_tn[p].y);
    }
    F.P = P;
    F.tau_lo = tlo;
    F.tau_hi = thi;
    F.nu_lo = vlo;
    F.nu_hi = vhi;
    if (npaths) npaths[blockIdx.x] = base;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// ---------------------------------------------------------------------------------------
// Plain form: one frame at a time, unfused kernels, scalars on the device
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_plain_init(const FrameDev* __restrict__ frames,
                                                       int f, const WorkItem* items, Bases B) {
  __shared__ float red[kWaves];
  const WorkItem wi = items[blockIdx.x];
  const FrameDev& F = frames[f];
  const FrameVecs V = frame_vecs(F, B);
  float acc = 0.f;
  const int64_t E = (int64_t)F.M * F.N;
  auto sink = [&](int q, float2 v) {
    F.c[q] = v;
    F.p0[q] = v;
    V.x[q] = make_float2(0.f, 0.f);
    acc = fmaf(v.x, v.x, acc);
    acc = fmaf(v.y, v.y, acc);
  };
  if (V.ybf16)
    band_apply<kRows, kPaths, true, false>(F, wi.l_begin, wi.l_end,
                                           SrcBf16{buf_rsrc(V.y, E * 4)}, sink);
  else
    band_apply<kRows, kPaths, true, false>(F, wi.l_begin, wi.l_end,
                                           SrcBuf{buf_rsrc(V.y, E * 8)}, sink);
  const float bs = block_sum(acc, red);
  if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
}

__global__ void k_plain_start(const FrameDev* __restrict__ frames, int f) {
  if (threadIdx.x != 0) return;
  const FrameDev& F = frames[f];
  const float cn0 = tile_sum(F.part_cc, F.T);
  FrameState s = *F.st;
  s.cn0 = cn0;
  s.cn_hist[0] = cn0;
  s.iter = 0;
  s.init = 1;
  s.rel = cn0 > 0.f ? 1.f : 0.f;
  s.status = cn0 > 0.f ? OTFS_FRAME_RUNNING
                       : (cn0 == 0.f ? OTFS_FRAME_CONVERGED : OTFS_FRAME_NONFINITE);
  *F.st = s;
}

__global__ __launch_bounds__(kBlock) void k_plain_H(const FrameDev* __restrict__ frames, int f,
                                                    const WorkItem* items) {
  const FrameDev& F = frames[f];
  if (F.st->status != OTFS_FRAME_RUNNING) return;
  const WorkItem wi = items[blockIdx.x];
  band_apply<kRows, kPaths, false, false>(
      F, wi.l_begin, wi.l_end, src_vec(F.p0, (int64_t)F.M * F.N),
      [&](int q, float2 v) { F.t[q] = v; });
}

__global__ __launch_bounds__(kBlock) void k_plain_HH(const FrameDev* __restrict__ frames, int f,
                                                     const WorkItem* items) {
  __shared__ float red[kWaves];
  const FrameDev& F = frames[f];
  if (F.st->status != OTFS_FRAME_RUNNING) return;
  const WorkItem wi = items[blockIdx.x];
  const float lam = F.lam;
  float acc = 0.f;
  band_apply<kRows, kPaths, true, false>(
      F, wi.l_begin, wi.l_end, src_vec(F.t, (int64_t)F.M * F.N),
      [&](int q, float2 v) {
        const float2 p = F.p0[q];
        const float2 a = axpyf(lam, p, v);
        F.a[q] = a;
        acc = fmaf(p.x, a.x, acc);
        acc = fmaf(p.y, a.y, acc);
      });
  const float bs = block_sum(acc, red);
  if (threadIdx.x == 0) F.part_pa[wi.tile] = bs;
}

__global__ __launch_bounds__(kBlock) void k_plain_update(const FrameDev* __restrict__ frames,
                                                         int f, const WorkItem* items, int xi,
                                                         Bases B) {
  __shared__ float red[kWaves];
  const FrameDev& F = frames[f];
  FrameState* st = F.st;
  if (st->status != OTFS_FRAME_RUNNING) return;
  const FrameVecs V = frame_vecs(F, B);
  const WorkItem wi = items[blockIdx.x];
  const float cn = st->cn_hist[(xi - 1) & 1];
  const float den = tile_sum(F.part_pa, F.T);
  const float alpha = cn / den;
  if (!(den > 0.f) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
      st->status = (isfinite(den) && isfinite(cn)) ? OTFS_FRAME_BREAKDOWN : OTFS_FRAME_NONFINITE;
    return;
  }
  float acc = 0.f;
  const int64_t q0 = (int64_t)wi.l_begin * F.M, q1 = (int64_t)wi.l_end * F.M;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock) {
    const float2 p = F.p0[q];
    V.x[q] = axpyf(alpha, p, V.x[q]);
    const float2 c = axpyf(-alpha, F.a[q], F.c[q]);
    F.c[q] = c;
    acc = fmaf(c.x, c.x, acc);
    acc = fmaf(c.y, c.y, acc);
  }
  const float bs = block_sum(acc, red);
  if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
}

__global__ __launch_bounds__(kBlock) void k_plain_dir(const FrameDev* __restrict__ frames,
                                                      int f, const WorkItem* items, int xi) {
  const FrameDev& F = frames[f];
  FrameState* st = F.st;
  if (st->status != OTFS_FRAME_RUNNING) return;
  const WorkItem wi = items[blockIdx.x];
  const float cn = st->cn_hist[(xi - 1) & 1];
  const float cn_new = tile_sum(F.part_cc, F.T);
  const float rel = sqrtf(cn_new / st->cn0);
  int status = OTFS_FRAME_RUNNING;
  if (!isfinite(cn_new))
    status = OTFS_FRAME_NONFINITE;
  else if (F.tol > 0.f && rel <= F.tol)
    status = OTFS_FRAME_CONVERGED;
  else if (xi >= F.max_iters)
    status = OTFS_FRAME_CAPPED;
  if (status == OTFS_FRAME_RUNNING) {
    const float beta = cn_new / cn;
    const int64_t q0 = (int64_t)wi.l_begin * F.M, q1 = (int64_t)wi.l_end * F.M;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock)
      F.p0[q] = axpyf(beta, F.p0[q], F.c[q]);
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->cn_hist[xi & 1] = cn_new;
    st->iter = xi;
    st->rel = rel;
    st->status = status;
  }
}

__global__ __launch_bounds__(kBlock) void k_plain_finish(const FrameDev* __restrict__ frames,
                                                         int f, const WorkItem* items, Bases B) {
  const FrameDev& F = frames[f];
  const FrameVecs V = frame_vecs(F, B);
  const WorkItem wi = items[blockIdx.x];
  const FrameState s = *F.st;
  const int status = s.status == OTFS_FRAME_RUNNING ? OTFS_FRAME_CAPPED : s.status;
  const bool dec = V.sym != nullptr && F.qside > 0;
  const int64_t q0 = (int64_t)wi.l_begin * F.M, q1 = (int64_t)wi.l_end * F.M;
  if (dec)
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock)
      V.sym[q] = decide(V.x[q], F.qscale, F.qside);
  if (blockIdx.x == 0 && threadIdx.x == 0 && V.stats) {
    otfs_frame_stats o{s.iter, s.rel, status, F.T};
    *V.stats = o;
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Static scratch of otfs_lmmse_cg_noalloc (callers that cannot allocate device memory):
// a plan workspace of at most kNoAllocBytes, one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel or a copy: it uses the
// device address that hipGetSymbolAddress returns, taken once per device with that device
// current.
// ---------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

hipError_t noalloc_scratch(int device, void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(mu);
  if (addr[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------------------
hipError_t launch_apply(bool adjoint, int sd, const FrameDev* frames, const WorkItem* items,
                        int nitems, const float2* in, float2* out, int lds_bytes, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g(nitems), b(kBlock);
  const int lb = sd != kDNone ? 0 : lds_bytes;
  if (lb > 0) {
    const void* fn = adjoint ? reinterpret_cast<const void*>(&k_apply<true, kDNone>)
                             : reinterpret_cast<const void*>(&k_apply<false, kDNone>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lb);
    if (e != hipSuccess) return e;
  }
  if (adjoint) {
    if (sd == kDBf16) hipLaunchKernelGGL((k_apply<true, kDBf16>), g, b, lb, s, frames, items, in, out);
    else if (sd == kDC64) hipLaunchKernelGGL((k_apply<true, kDC64>), g, b, lb, s, frames, items, in, out);
    else hipLaunchKernelGGL((k_apply<true, kDNone>), g, b, lb, s, frames, items, in, out);
  } else {
    if (sd == kDBf16) hipLaunchKernelGGL((k_apply<false, kDBf16>), g, b, lb, s, frames, items, in, out);
    else if (sd == kDC64) hipLaunchKernelGGL((k_apply<false, kDC64>), g, b, lb, s, frames, items, in, out);
    else hipLaunchKernelGGL((k_apply<false, kDNone>), g, b, lb, s, frames, items, in, out);
  }
  return hipGetLastError();
}

hipError_t launch_reset(const FrameDev* frames, int nframes, unsigned* abort_flag,
                        unsigned* qhead, int ngroups, hipStream_t s) {
  const int n = nframes > ngroups ? nframes : ngroups;
  if (n <= 0) return hipSuccess;
  const int grid = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(kBlock), 0, s, frames, nframes, abort_flag,
                     qhead, ngroups);
  return hipGetLastError();
}

hipError_t launch_step_reset(const FrameDev* frames, int nframes, unsigned* abort_flag,
                             unsigned* qhead, int ngroups, hipStream_t s) {
  const int n = nframes > ngroups ? nframes : ngroups;
  if (n <= 0) return hipSuccess;
  const int grid = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_step_reset, dim3(grid), dim3(kBlock), 0, s, frames, nframes, abort_flag,
                     qhead, ngroups);
  return hipGetLastError();
}

// ticks of the wall clock that the kernels' bounded waits read (s_memrealtime)
static uint64_t wallclock_ticks_per_us() {
  static uint64_t per_us = 0;
  if (per_us == 0) {
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    per_us = std::max<uint64_t>(1, (uint64_t)khz / 1000ull);
  }
  return per_us;
}
// wait_us < 0: the default bound of 20 s; 0: a wait gives up at its first unsatisfied poll
static uint64_t wait_ticks(int64_t wait_us) {
  if (wait_us < 0) wait_us = 20ll * 1000 * 1000;
  return (uint64_t)wait_us * wallclock_ticks_per_us();
}

template <int SD, int KIND>
static void launch_fused_t(const FrameDev* frames, const WorkItem* items, const int32_t* qitems,
                           const int2* qrange, unsigned* qhead, int ngroups, int grid, int budget,
                           const Bases& bases, const LaunchCtx& L, int lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_fused<SD, KIND>), dim3(grid), dim3(kBlock), lds_bytes, s, frames, items,
                     qitems, qrange, qhead, ngroups, budget, bases, L);
}

// the instantiation of a launch kind: only the direct kind reads a stored D (the host
// guarantees it)
static const void* fused_fn(int kind, int sd) {
  switch (kind) {
    case kKindResident: return reinterpret_cast<const void*>(&k_cg_fused<kDNone, kKindResident>);
    case kKindWindowed: return reinterpret_cast<const void*>(&k_cg_fused<kDNone, kKindWindowed>);
    case kKindDirectFD: return reinterpret_cast<const void*>(&k_cg_fused<kDNone, kKindDirectFD>);
    case kKindStaged: return reinterpret_cast<const void*>(&k_cg_fused<kDNone, kKindStaged>);
    case kKindLds: return reinterpret_cast<const void*>(&k_cg_fused<kDNone, kKindLds>);
    default: break;
  }
  if (sd == kDBf16) return reinterpret_cast<const void*>(&k_cg_fused<kDBf16, kKindDirect>);
  if (sd == kDC64) return reinterpret_cast<const void*>(&k_cg_fused<kDC64, kKindDirect>);
  return reinterpret_cast<const void*>(&k_cg_fused<kDNone, kKindDirect>);
}

hipError_t launch_cg_fused(int kind, int sd, const FrameDev* frames, const WorkItem* items,
                           const int32_t* qitems, const int2* qrange, unsigned* qhead, int ngroups,
                           int grid, int budget, Bases bases, bool xcd_local, unsigned* abort_flag,
                           int lds_bytes, int64_t wait_us, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (kind != kKindDirect && sd != kDNone) return hipErrorInvalidValue;
  LaunchCtx L{abort_flag, wait_ticks(wait_us), xcd_local ? 1 : 0};
  if (kind == kKindWindowed || kind == kKindStaged || kind == kKindLds) {
    hipError_t e = hipFuncSetAttribute(fused_fn(kind, sd), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       lds_bytes);
    if (e != hipSuccess) return e;
  }
  switch (kind) {
    case kKindResident:
      launch_fused_t<kDNone, kKindResident>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, lds_bytes, s);
      break;
    case kKindWindowed:
      launch_fused_t<kDNone, kKindWindowed>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, lds_bytes, s);
      break;
    case kKindDirectFD:
      launch_fused_t<kDNone, kKindDirectFD>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, 0, s);
      break;
    case kKindStaged:
      launch_fused_t<kDNone, kKindStaged>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, lds_bytes, s);
      break;
    case kKindLds:
      launch_fused_t<kDNone, kKindLds>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, lds_bytes, s);
      break;
    default:
      if (sd == kDBf16)
        launch_fused_t<kDBf16, kKindDirect>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, 0, s);
      else if (sd == kDC64)
        launch_fused_t<kDC64, kKindDirect>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, 0, s);
      else
        launch_fused_t<kDNone, kKindDirect>(frames, items, qitems, qrange, qhead, ngroups, grid, budget, bases, L, 0, s);
  }
  return hipGetLastError();
}

hipError_t launch_refresh(const FrameDev* frames, const WorkItem* items, int nitems, Bases bases,
                          unsigned* qhead, int nq, int lds_bytes, int nxcd, hipStream_t s) {
  if (nitems <= 0 || nq > kBlock || lds_bytes < 0 || nxcd < 1) return hipErrorInvalidValue;
  if (lds_bytes > 0) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_refresh_u),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_refresh_c),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_refresh_u, dim3(nitems), dim3(kBlock), lds_bytes, s, frames, items, bases,
                     qhead, nq, lds_bytes, nxcd);
  hipLaunchKernelGGL(k_refresh_c, dim3(nitems), dim3(kBlock), lds_bytes, s, frames, items, bases,
                     lds_bytes, nxcd);
  return hipGetLastError();
}

int fused_blocks_per_cu(int kind, int sd, int lds_bytes) {
  int n = 0;
  if (kind == kKindDirect || kind == kKindDirectFD) lds_bytes = 0;
  const void* fn = fused_fn(kind, sd);
  if (lds_bytes > 0)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kBlock, lds_bytes) != hipSuccess)
    n = 0;
  return n;
}

hipError_t launch_xcc_probe(int* out, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_xcc_probe, dim3(nblocks), dim3(64), 0, s, out);
  return hipGetLastError();
}

hipError_t launch_plain_frame(const FrameDev* frames_dev, int f, const WorkItem* items_dev,
                              int item_begin, int ntiles, int max_iters, Bases B, hipStream_t s) {
  const WorkItem* it = items_dev + item_begin;
  const dim3 g(ntiles), b(kBlock);
  hipLaunchKernelGGL(k_plain_init, g, b, 0, s, frames_dev, f, it, B);
  hipLaunchKernelGGL(k_plain_start, dim3(1), dim3(64), 0, s, frames_dev, f);
  for (int xi = 1; xi <= max_iters; ++xi) {
    hipLaunchKernelGGL(k_plain_H, g, b, 0, s, frames_dev, f, it);
    hipLaunchKernelGGL(k_plain_HH, g, b, 0, s, frames_dev, f, it);
    hipLaunchKernelGGL(k_plain_update, g, b, 0, s, frames_dev, f, it, xi, B);
    hipLaunchKernelGGL(k_plain_dir, g, b, 0, s, frames_dev, f, it, xi);
  }
  hipLaunchKernelGGL(k_plain_finish, g, b, 0, s, frames_dev, f, it, B);
  return hipGetLastError();
}

hipError_t launch_bit_errors(const FrameDev* frames, const WorkItem* items, int nitems,
                             const uint8_t* sym, const uint8_t* tx, unsigned long long* errs,
                             int nframes, bool clear, hipStream_t s) {
  if (clear && nframes > 0)
    hipLaunchKernelGGL(k_fill_u64, dim3((nframes + 255) / 256), dim3(256), 0, s, errs,
                       (int64_t)nframes);
  if (nitems > 0)
    hipLaunchKernelGGL(k_bit_errors, dim3(nitems), dim3(kBlock), 0, s, frames, items, sym, tx, errs);
  return hipGetLastError();
}

hipError_t launch_trace_errors(const FrameDev* frames, const WorkItem* items, int nitems, Bases B,
                               const uint8_t* tx, unsigned long long* errs, hipStream_t s) {
  if (nitems > 0)
    hipLaunchKernelGGL(k_trace_errors, dim3(nitems), dim3(kBlock), 0, s, frames, items, B, tx, errs);
  return hipGetLastError();
}

// Gather of result regions into one staging buffer (the serving loop's result copy): one
// workgroup per segment, 16-byte vector copies, the last bytes of a segment one by one.
__global__ __launch_bounds__(256) void k_gather_segments(const CopySeg* __restrict__ segs,
                                                         unsigned char* __restrict__ dst) {
  const CopySeg sg = segs[blockIdx.x];
  const uint64_t n16 = sg.bytes / 16;
  const uint4* s4 = reinterpret_cast<const uint4*>(sg.src);
  uint4* d4 = reinterpret_cast<uint4*>(dst + sg.dst);
  for (uint64_t i = threadIdx.x; i < n16; i += blockDim.x) d4[i] = s4[i];
  for (uint64_t i = n16 * 16 + threadIdx.x; i < sg.bytes; i += blockDim.x)
    dst[sg.dst + i] = sg.src[i];
}

hipError_t launch_gather_segments(const CopySeg* segs, int nseg, unsigned char* dst,
                                  hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_segments, dim3((unsigned)nseg), dim3(256), 0, s, segs, dst);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       s, p, n);
  return hipGetLastError();
}

hipError_t launch_pilot_paths(FrameDev* frames, int nframes, const float2* ypilot, float theta,
                              int32_t* npaths, hipStream_t s) {
  if (nframes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pilot_paths, dim3(nframes), dim3(kBlock), 0, s, frames, ypilot, theta,
                     npaths);
  return hipGetLastError();
}

hipError_t launch_build_d(int sd, const FrameDev* frames, const WorkItem* items, int nitems,
                          hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (sd == kDC64)
    hipLaunchKernelGGL(k_build_d<kDC64>, dim3(nitems), dim3(kBlock), 0, s, frames, items);
  else
    hipLaunchKernelGGL(k_build_d<kDBf16>, dim3(nitems), dim3(kBlock), 0, s, frames, items);
  return hipGetLastError();
}

}  // namespace otfs
