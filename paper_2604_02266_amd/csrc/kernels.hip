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

#include "otfs_internal.h"

namespace otfs {
namespace {

// ---------------------------------------------------------------------------------------
// small complex helpers
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cmacf(float2& acc, float2 c, float2 v) {
  acc.x = fmaf(c.x, v.x, acc.x);
  acc.x = fmaf(-c.y, v.y, acc.x);
  acc.y = fmaf(c.x, v.y, acc.y);
  acc.y = fmaf(c.y, v.x, acc.y);
}
__device__ __forceinline__ double2 cmuld(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
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
__device__ float block_sum(float v, float* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) s += red[i];
  __syncthreads();
  return s;
}
__device__ double block_sum_d(double v, double* red) {
  v = wave_sum_d(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) s += red[i];
  __syncthreads();
  return s;
}
// sum of the T per-tile partials of a frame, in tile order, by every thread
__device__ __forceinline__ double tile_sum(const float* part, int T) {
  double s = 0.0;
  for (int i = 0; i < T; ++i) s += (double)part[i];
  return s;
}
__device__ __forceinline__ double tile_sum_d(const double* part, int T) {
  double s = 0.0;
  for (int i = 0; i < T; ++i) s += part[i];
  return s;
}

// ---------------------------------------------------------------------------------------
// per-frame barrier among the T workgroups that share a frame
// ---------------------------------------------------------------------------------------
// Every thread releases its own stores at agent scope (the L2s of different XCDs are not
// coherent), the workgroup meets, one lane counts the arrival and waits for all T arrivals
// of this barrier round, the workgroup meets again and every thread acquires.  The wait is
// bounded: after `timeout` ticks of the 100 MHz wall clock, or when another workgroup has
// raised the launch-wide abort flag, it gives up and reports failure.
__device__ bool frame_barrier(unsigned* ctr, unsigned target, unsigned* abort_flag,
                              uint64_t timeout, int* sflag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          wall_clock64() - t0 > timeout) {
        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
    *sflag = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *sflag != 0;
}

// ---------------------------------------------------------------------------------------
// Tiled operator applications.  src(i) returns element i (frame-local index) of the
// vector being multiplied; sink(q, v) receives output element q of the band.  Threads
// with nothing to do return early; callers put block-wide work after the call.
// ---------------------------------------------------------------------------------------
template <int PMAX, bool STORED, class Src, class Sink>
__device__ __forceinline__ void apply_fwd(const FrameDev& F, int lb, int le, Src src,
                                          Sink sink) {
  const int M = F.M, N = F.N, P = F.P;
  const int TX = M < kBlock ? M : kBlock;
  const int TY = kBlock / TX;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  if (ty >= TY) return;
  const int64_t E = (int64_t)M * N;
  for (int k = tx; k < M; k += TX) {
    float2 cf[PMAX];
    int ks[PMAX], nw[PMAX], nu[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
      if (p < P) {
        const int2 tn = F.paths[p];
        const int K = k - tn.x;                        // raw source delay
        const int n = K < 0 ? -1 : (K >= M ? 1 : 0);   // delay wrap count
        ks[p] = K - n * M;
        nw[p] = n;
        nu[p] = tn.y;
        if (!STORED) cf[p] = F.rtab[p * M + k];
      }
    }
    for (int l = lb + ty; l < le; l += TY) {
      float2 acc = make_float2(0.f, 0.f);
      const int q = l * M + k;
#pragma unroll
      for (int p = 0; p < PMAX; ++p) {
        if (p < P) {
          int ls = l - nu[p];
          ls += ls < 0 ? N : 0;
          ls -= ls >= N ? N : 0;
          const float2 v = src(ls * M + ks[p]);
          float2 c;
          if (STORED) {
            c = bf16x2_to_f2(F.dtab[(int64_t)p * E + q]);
          } else {
            c = cf[p];
            if (nw[p] != 0) {
              float2 w = F.wtab[ls];
              if (nw[p] < 0) w.y = -w.y;
              c = cmulf(c, w);
            }
          }
          cmacf(acc, c, v);
        }
      }
      sink(q, acc);
    }
  }
}

template <int PMAX, bool STORED, class Src, class Sink>
__device__ __forceinline__ void apply_adj(const FrameDev& F, int lb, int le, Src src,
                                          Sink sink) {
  const int M = F.M, N = F.N, P = F.P;
  const int TX = M < kBlock ? M : kBlock;
  const int TY = kBlock / TX;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  if (ty >= TY) return;
  const int64_t E = (int64_t)M * N;
  for (int k = tx; k < M; k += TX) {
    float2 cf[PMAX];
    int kq[PMAX], ww[PMAX], nu[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
      if (p < P) {
        const int2 tn = F.paths[p];
        const int Kq = k + tn.x;
        const int w = Kq < 0 ? -1 : (Kq >= M ? 1 : 0);   // the gathered row wraps by -w
        kq[p] = Kq - w * M;
        ww[p] = w;
        nu[p] = tn.y;
        if (!STORED) {
          const float2 r = F.rtab[p * M + kq[p]];
          cf[p] = make_float2(r.x, -r.y);
        }
      }
    }
    for (int l = lb + ty; l < le; l += TY) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int p = 0; p < PMAX; ++p) {
        if (p < P) {
          int lq = l + nu[p];
          lq += lq < 0 ? N : 0;
          lq -= lq >= N ? N : 0;
          const int qs = lq * M + kq[p];
          const float2 v = src(qs);
          float2 c;
          if (STORED) {
            const float2 d = bf16x2_to_f2(F.dtab[(int64_t)p * E + qs]);
            c = make_float2(d.x, -d.y);
          } else {
            c = cf[p];
            if (ww[p] != 0) {        // conj(W[l]^{-w}) = W[l]^{w}
              float2 w = F.wtab[l];
              if (ww[p] < 0) w.y = -w.y;
              c = cmulf(c, w);
            }
          }
          cmacf(acc, c, v);
        }
      }
      sink(l * M + k, acc);
    }
  }
}

// FP64 versions (coefficients from the FP64 tables) for the true-residual refresh.
template <int PMAX, class Src, class Sink>
__device__ __forceinline__ void apply_fwd64(const FrameDev& F, int lb, int le, Src src,
                                            Sink sink) {
  const int M = F.M, N = F.N, P = F.P;
  const int TX = M < kBlock ? M : kBlock;
  const int TY = kBlock / TX;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  if (ty >= TY) return;
  for (int k = tx; k < M; k += TX) {
    for (int l = lb + ty; l < le; l += TY) {
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < PMAX; ++p) {
        if (p < P) {
          const int2 tn = F.paths[p];
          const int K = k - tn.x;
          const int n = K < 0 ? -1 : (K >= M ? 1 : 0);
          int ls = l - tn.y;
          ls += ls < 0 ? N : 0;
          ls -= ls >= N ? N : 0;
          const double2 v = src(ls * M + (K - n * M));
          double2 c = F.rtab64[p * M + k];
          if (n != 0) {
            double2 w = F.wtab64[ls];
            if (n < 0) w.y = -w.y;
            c = cmuld(c, w);
          }
          cmacd(acc, c, v);
        }
      }
      sink(l * M + k, acc);
    }
  }
}

template <int PMAX, class Src, class Sink>
__device__ __forceinline__ void apply_adj64(const FrameDev& F, int lb, int le, Src src,
                                            Sink sink) {
  const int M = F.M, N = F.N, P = F.P;
  const int TX = M < kBlock ? M : kBlock;
  const int TY = kBlock / TX;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  if (ty >= TY) return;
  for (int k = tx; k < M; k += TX) {
    for (int l = lb + ty; l < le; l += TY) {
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int p = 0; p < PMAX; ++p) {
        if (p < P) {
          const int2 tn = F.paths[p];
          const int Kq = k + tn.x;
          const int w = Kq < 0 ? -1 : (Kq >= M ? 1 : 0);
          const int kq = Kq - w * M;
          int lq = l + tn.y;
          lq += lq < 0 ? N : 0;
          lq -= lq >= N ? N : 0;
          const double2 v = src(lq * M + kq);
          const double2 r = F.rtab64[p * M + kq];
          double2 c = make_double2(r.x, -r.y);
          if (w != 0) {
            double2 wl = F.wtab64[l];
            if (w < 0) wl.y = -wl.y;
            c = cmuld(c, wl);
          }
          cmacd(acc, c, v);
        }
      }
      sink(l * M + k, acc);
    }
  }
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
__device__ void finish_tile(const FrameDev& F, const WorkItem& wi, const FrameVecs& V,
                            const FrameState& s, const float2* pcur, bool xpending,
                            int status) {
  const int M = F.M;
  const int64_t q0 = (int64_t)wi.l_begin * M, q1 = (int64_t)wi.l_end * M;
  const bool dec = V.sym != nullptr && F.qside > 0;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock) {
    float2 xv = V.x[q];
    if (xpending) {
      xv = axpyf(s.alpha, pcur[q], xv);
      V.x[q] = xv;
    }
    if (dec) V.sym[q] = decide(xv, F.qscale, F.qside);
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
//   the finish).  Every k-th iteration (refresh_every) c is replaced by the FP64 true
//   residual H^H (y - H x) - lam x (two more passes, two more barriers).
// ---------------------------------------------------------------------------------------
struct LaunchCtx {
  unsigned* abort_flag;
  uint64_t timeout;
};

template <int PMAX, bool STORED>
__device__ void cg_item(const FrameDev& F, const WorkItem& wi, int budget, const Bases& B,
                        const LaunchCtx& L, float* red, double* redd, int* sflag) {
  const FrameVecs V = frame_vecs(F, B);
  FrameState s = *F.st;
  if (s.status != OTFS_FRAME_RUNNING) return;
  const int M = F.M, T = F.T;
  const int lb = wi.l_begin, le = wi.l_end;
  const int64_t q0 = (int64_t)lb * M, q1 = (int64_t)le * M;
  const float lam = F.lam;
  unsigned nbar = 0;
  auto bar = [&]() -> bool {
    if (T == 1) {
      __syncthreads();
      return true;
    }
    nbar += (unsigned)T;
    return frame_barrier(F.bar, nbar, L.abort_flag, L.timeout, sflag);
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

  // ---- b = H^H y; x = 0; c = p = b; c_norm_0 = ||b||^2 (Algorithm 1, first line) ----
  if (!s.init) {
    float acc = 0.f;
    apply_adj<PMAX, STORED>(
        F, lb, le, [&](int i) { return load_y(V.y, i, V.ybf16); },
        [&](int q, float2 v) {
          F.c[q] = v;
          F.p0[q] = v;
          V.x[q] = make_float2(0.f, 0.f);
          acc = fmaf(v.x, v.x, acc);
          acc = fmaf(v.y, v.y, acc);
        });
    const float bs = block_sum(acc, red);
    if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
    if (!bar()) return fail_timeout();
    const float cn0 = (float)tile_sum(F.part_cc, T);
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
    float2* pold = s.pbuf ? F.p1 : F.p0;
    const bool dirp = (s.pending & 2) != 0, xp = (s.pending & 1) != 0;
    float2* pnew = dirp ? (s.pbuf ? F.p0 : F.p1) : pold;
    const float al = s.alpha, be = s.beta;

    // ---- A: deferred updates of the band, t = H p ----
    if (dirp) {
      apply_fwd<PMAX, STORED>(
          F, lb, le, [&](int i) { return axpyf(be, pold[i], F.c[i]); },
          [&](int q, float2 v) {
            F.t[q] = v;
            const float2 po = pold[q];
            pnew[q] = axpyf(be, po, F.c[q]);
            if (xp) V.x[q] = axpyf(al, po, V.x[q]);
          });
    } else {
      apply_fwd<PMAX, STORED>(
          F, lb, le, [&](int i) { return pold[i]; },
          [&](int q, float2 v) {
            F.t[q] = v;
            if (xp) V.x[q] = axpyf(al, pold[q], V.x[q]);
          });
    }
    if (!bar()) return fail_timeout();

    // ---- B: a = H^H t + lam p, partial Re(p^H a) ----
    {
      float acc = 0.f;
      apply_adj<PMAX, STORED>(
          F, lb, le, [&](int i) { return F.t[i]; },
          [&](int q, float2 v) {
            const float2 p = pnew[q];
            const float2 a = axpyf(lam, p, v);
            F.a[q] = a;
            acc = fmaf(p.x, a.x, acc);
            acc = fmaf(p.y, a.y, acc);
          });
      const float bs = block_sum(acc, red);
      if (threadIdx.x == 0) F.part_pa[wi.tile] = bs;
    }
    if (!bar()) return fail_timeout();
    s.pbuf = (pnew == F.p1) ? 1 : 0;
    s.pending = 0;                                   // both deferred updates are applied

    const float den = (float)tile_sum(F.part_pa, T);
    const float alpha = s.cn / den;
    if (!(den > 0.f) || !isfinite(alpha)) {          // x already holds x_{xi-1}
      const int st = (isfinite(den) && isfinite(s.cn)) ? OTFS_FRAME_BREAKDOWN
                                                        : OTFS_FRAME_NONFINITE;
      return finish_tile(F, wi, V, s, pnew, false, st);
    }

    // ---- C: c -= alpha a, partial ||c||^2 ----
    {
      float acc = 0.f;
      for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock) {
        const float2 c = axpyf(-alpha, F.a[q], F.c[q]);
        F.c[q] = c;
        acc = fmaf(c.x, c.x, acc);
        acc = fmaf(c.y, c.y, acc);
      }
      const float bs = block_sum(acc, red);
      if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
    }
    if (!bar()) return fail_timeout();
    float cn_new = (float)tile_sum(F.part_cc, T);
    s.iter = xi;
    s.alpha = alpha;
    bool xpend = true;                               // x += alpha p_new still to do

    // ---- FP64 true-residual refresh ----
    if (F.refresh_every > 0 && xi % F.refresh_every == 0 && xi < F.max_iters &&
        isfinite(cn_new)) {
      // R1: u = y - H (x + alpha p) in FP64 (x itself is not written while others read it)
      apply_fwd64<PMAX>(
          F, lb, le,
          [&](int i) {
            const float2 xv = axpyf(alpha, pnew[i], V.x[i]);
            return make_double2((double)xv.x, (double)xv.y);
          },
          [&](int q, double2 v) {
            const float2 yv = load_y(V.y, q, V.ybf16);
            F.u[q] = make_double2((double)yv.x - v.x, (double)yv.y - v.y);
          });
      if (!bar()) return fail_timeout();
      // R2: c = H^H u - lam x, with x += alpha p applied here
      double acc = 0.0;
      apply_adj64<PMAX>(
          F, lb, le, [&](int i) { return F.u[i]; },
          [&](int q, double2 v) {
            const float2 xn = axpyf(alpha, pnew[q], V.x[q]);
            V.x[q] = xn;
            const float2 cf = make_float2((float)(v.x - (double)lam * (double)xn.x),
                                          (float)(v.y - (double)lam * (double)xn.y));
            F.c[q] = cf;
            acc = fma((double)cf.x, (double)cf.x, acc);
            acc = fma((double)cf.y, (double)cf.y, acc);
          });
      const double bs = block_sum_d(acc, redd);
      if (threadIdx.x == 0) F.part_d[wi.tile] = bs;
      if (!bar()) return fail_timeout();
      cn_new = (float)tile_sum_d(F.part_d, T);
      xpend = false;
    }

    s.rel = sqrtf(cn_new / s.cn0);
    if (!isfinite(cn_new)) return finish_tile(F, wi, V, s, pnew, xpend, OTFS_FRAME_NONFINITE);
    if (F.tol > 0.f && s.rel <= F.tol)
      return finish_tile(F, wi, V, s, pnew, xpend, OTFS_FRAME_CONVERGED);
    if (xi >= F.max_iters) return finish_tile(F, wi, V, s, pnew, xpend, OTFS_FRAME_CAPPED);
    s.beta = cn_new / s.cn;
    s.cn = cn_new;
    s.pending = (xpend ? 1 : 0) | 2;
  }
  // iteration budget of this launch used up: keep the state for the next launch
  if (wi.tile == 0 && threadIdx.x == 0) *F.st = s;
}

template <int PMAX>
__global__ __launch_bounds__(kBlock) void k_cg_fused(const FrameDev* __restrict__ frames,
                                                     const WorkItem* __restrict__ items,
                                                     const int32_t* __restrict__ sched,
                                                     const int2* __restrict__ ranges,
                                                     int budget, Bases B, LaunchCtx L) {
  __shared__ float red[kWaves];
  __shared__ double redd[kWaves];
  __shared__ int sflag;
  const int2 r = ranges[blockIdx.x];
  for (int j = r.x; j < r.y; ++j) {
    const WorkItem wi = items[sched[j]];
    const FrameDev F = frames[wi.frame];
    if (F.dtab)
      cg_item<PMAX, true>(F, wi, budget, B, L, red, redd, &sflag);
    else
      cg_item<PMAX, false>(F, wi, budget, B, L, red, redd, &sflag);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// standalone operator applications (one workgroup per tile)
// ---------------------------------------------------------------------------------------
template <int PMAX, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_apply(const FrameDev* __restrict__ frames,
                                                  const WorkItem* __restrict__ items,
                                                  const float2* __restrict__ in,
                                                  float2* __restrict__ out) {
  const WorkItem wi = items[blockIdx.x];
  const FrameDev F = frames[wi.frame];
  const float2* src = in + F.off;
  float2* dst = out + F.off;
  auto ld = [&](int i) { return src[i]; };
  auto st = [&](int q, float2 v) { dst[q] = v; };
  if (F.dtab) {
    if (ADJ) apply_adj<PMAX, true>(F, wi.l_begin, wi.l_end, ld, st);
    else apply_fwd<PMAX, true>(F, wi.l_begin, wi.l_end, ld, st);
  } else {
    if (ADJ) apply_adj<PMAX, false>(F, wi.l_begin, wi.l_end, ld, st);
    else apply_fwd<PMAX, false>(F, wi.l_begin, wi.l_end, ld, st);
  }
}

__global__ void k_reset(const FrameDev* __restrict__ frames, int nframes, unsigned* abort_flag) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && abort_flag) *abort_flag = 0u;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nframes; i += gridDim.x * blockDim.x) {
    const FrameDev& F = frames[i];
    *F.bar = 0u;
    FrameState s;
    s.iter = 0;
    s.status = OTFS_FRAME_RUNNING;
    s.pbuf = 0;
    s.pending = 0;
    s.cn = s.cn0 = s.alpha = s.beta = s.rel = 0.f;
    s.init = 0;
    s.cn_hist[0] = s.cn_hist[1] = 0.f;
    *F.st = s;
  }
}

// Stored coefficients D_{p,q} (Eq. D_definition) of every frame as bf16 pairs.
template <int PMAX>
__global__ __launch_bounds__(kBlock) void k_build_d(const FrameDev* __restrict__ frames,
                                                    const WorkItem* __restrict__ items) {
  const WorkItem wi = items[blockIdx.x];
  const FrameDev F = frames[wi.frame];
  const int M = F.M, N = F.N;
  const int64_t E = (int64_t)M * N;
  uint32_t* d = const_cast<uint32_t*>(F.dtab);
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
      d[p * E + q] = f32_to_bf16(c.x) | (f32_to_bf16(c.y) << 16);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Plain form: one frame at a time, unfused kernels, scalars on the device
// ---------------------------------------------------------------------------------------
template <int PMAX>
__global__ __launch_bounds__(kBlock) void k_plain_init(const FrameDev* __restrict__ frames,
                                                       int f, const WorkItem* items, Bases B) {
  __shared__ float red[kWaves];
  const WorkItem wi = items[blockIdx.x];
  const FrameDev F = frames[f];
  const FrameVecs V = frame_vecs(F, B);
  float acc = 0.f;
  apply_adj<PMAX, false>(
      F, wi.l_begin, wi.l_end, [&](int i) { return load_y(V.y, i, V.ybf16); },
      [&](int q, float2 v) {
        F.c[q] = v;
        F.p0[q] = v;
        V.x[q] = make_float2(0.f, 0.f);
        acc = fmaf(v.x, v.x, acc);
        acc = fmaf(v.y, v.y, acc);
      });
  const float bs = block_sum(acc, red);
  if (threadIdx.x == 0) F.part_cc[wi.tile] = bs;
}

__global__ void k_plain_start(const FrameDev* __restrict__ frames, int f) {
  if (threadIdx.x != 0) return;
  const FrameDev F = frames[f];
  const float cn0 = (float)tile_sum(F.part_cc, F.T);
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

template <int PMAX>
__global__ __launch_bounds__(kBlock) void k_plain_H(const FrameDev* __restrict__ frames, int f,
                                                    const WorkItem* items) {
  const FrameDev F = frames[f];
  if (F.st->status != OTFS_FRAME_RUNNING) return;
  const WorkItem wi = items[blockIdx.x];
  apply_fwd<PMAX, false>(
      F, wi.l_begin, wi.l_end, [&](int i) { return F.p0[i]; },
      [&](int q, float2 v) { F.t[q] = v; });
}

template <int PMAX>
__global__ __launch_bounds__(kBlock) void k_plain_HH(const FrameDev* __restrict__ frames, int f,
                                                     const WorkItem* items) {
  __shared__ float red[kWaves];
  const FrameDev F = frames[f];
  if (F.st->status != OTFS_FRAME_RUNNING) return;
  const WorkItem wi = items[blockIdx.x];
  const float lam = F.lam;
  float acc = 0.f;
  apply_adj<PMAX, false>(
      F, wi.l_begin, wi.l_end, [&](int i) { return F.t[i]; },
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
  const FrameDev F = frames[f];
  FrameState* st = F.st;
  if (st->status != OTFS_FRAME_RUNNING) return;
  const FrameVecs V = frame_vecs(F, B);
  const WorkItem wi = items[blockIdx.x];
  const float cn = st->cn_hist[(xi - 1) & 1];
  const float den = (float)tile_sum(F.part_pa, F.T);
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
  const FrameDev F = frames[f];
  FrameState* st = F.st;
  if (st->status != OTFS_FRAME_RUNNING) return;
  const WorkItem wi = items[blockIdx.x];
  const float cn = st->cn_hist[(xi - 1) & 1];
  const float cn_new = (float)tile_sum(F.part_cc, F.T);
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
  const FrameDev F = frames[f];
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
// host-side launchers
// ---------------------------------------------------------------------------------------
int pmax_bucket(int max_paths) {
  if (max_paths <= 4) return 4;
  if (max_paths <= 8) return 8;
  if (max_paths <= 16) return 16;
  if (max_paths <= 32) return 32;
  return 64;
}

#define OTFS_PMAX_SWITCH(pm, BODY)            \
  switch (pm) {                               \
    case 4: { constexpr int PM = 4; BODY; } break;   \
    case 8: { constexpr int PM = 8; BODY; } break;   \
    case 16: { constexpr int PM = 16; BODY; } break; \
    case 32: { constexpr int PM = 32; BODY; } break; \
    default: { constexpr int PM = 64; BODY; } break; \
  }

hipError_t launch_apply(bool adjoint, int pmax, const FrameDev* frames, const WorkItem* items,
                        int nitems, const float2* in, float2* out, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  OTFS_PMAX_SWITCH(pmax, {
    if (adjoint)
      hipLaunchKernelGGL((k_apply<PM, true>), dim3(nitems), dim3(kBlock), 0, s, frames, items, in, out);
    else
      hipLaunchKernelGGL((k_apply<PM, false>), dim3(nitems), dim3(kBlock), 0, s, frames, items, in, out);
  });
  return hipGetLastError();
}

hipError_t launch_reset(const FrameDev* frames, int nframes, unsigned* abort_flag, hipStream_t s) {
  if (nframes <= 0) return hipSuccess;
  const int grid = (nframes + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(kBlock), 0, s, frames, nframes, abort_flag);
  return hipGetLastError();
}

static uint64_t wallclock_timeout_ticks() {
  static uint64_t ticks = 0;
  if (ticks == 0) {
    int dev = 0, khz = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
      khz = 100000;
    ticks = (uint64_t)khz * 1000ull * 20ull;   // 20 s
  }
  return ticks;
}

hipError_t launch_cg_fused(int pmax, const FrameDev* frames, const WorkItem* items,
                           const int32_t* sched, const int2* ranges, int grid, int budget,
                           Bases bases, hipStream_t s, unsigned* abort_flag) {
  if (grid <= 0) return hipSuccess;
  LaunchCtx L{abort_flag, wallclock_timeout_ticks()};
  OTFS_PMAX_SWITCH(pmax, {
    hipLaunchKernelGGL((k_cg_fused<PM>), dim3(grid), dim3(kBlock), 0, s, frames, items, sched,
                       ranges, budget, bases, L);
  });
  return hipGetLastError();
}

int fused_blocks_per_cu(int pmax) {
  int n = 0;
  OTFS_PMAX_SWITCH(pmax, {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_cg_fused<PM>), kBlock, 0) != hipSuccess)
      n = 0;
  });
  return n;
}

hipError_t launch_plain_frame(int pmax, const FrameDev* frames_dev, int f,
                              const WorkItem* items_dev, int item_begin, int ntiles,
                              int max_iters, Bases B, hipStream_t s) {
  const WorkItem* it = items_dev + item_begin;
  const dim3 g(ntiles), b(kBlock);
  OTFS_PMAX_SWITCH(pmax, {
    hipLaunchKernelGGL((k_plain_init<PM>), g, b, 0, s, frames_dev, f, it, B);
    hipLaunchKernelGGL(k_plain_start, dim3(1), dim3(64), 0, s, frames_dev, f);
    for (int xi = 1; xi <= max_iters; ++xi) {
      hipLaunchKernelGGL((k_plain_H<PM>), g, b, 0, s, frames_dev, f, it);
      hipLaunchKernelGGL((k_plain_HH<PM>), g, b, 0, s, frames_dev, f, it);
      hipLaunchKernelGGL(k_plain_update, g, b, 0, s, frames_dev, f, it, xi, B);
      hipLaunchKernelGGL(k_plain_dir, g, b, 0, s, frames_dev, f, it, xi);
    }
    hipLaunchKernelGGL(k_plain_finish, g, b, 0, s, frames_dev, f, it, B);
  });
  return hipGetLastError();
}

hipError_t launch_build_d(int pmax, const FrameDev* frames, const WorkItem* items, int nitems,
                          hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  OTFS_PMAX_SWITCH(pmax, {
    hipLaunchKernelGGL((k_build_d<PM>), dim3(nitems), dim3(kBlock), 0, s, frames, items);
  });
  return hipGetLastError();
}

}  // namespace otfs
