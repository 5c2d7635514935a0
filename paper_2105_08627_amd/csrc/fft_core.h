// Device building blocks of the FFT passes (gfx950): complex helpers, radix
// 2/3/4/8 DFTs, LDS accessors, the mixed-radix Stockham stage, compile-time
// plans and the persistent item loop.
//
// Stockham stage with radix R after Ns previous points (natural order out):
//   in  v_r = src[j + r L/R],  twiddle  v_r *= w_L^(r (j mod Ns) L/(Ns R))
//   R-point DFT, out dst[(j / Ns) Ns R + (j mod Ns) + r Ns].
#pragma once

#include <type_traits>
#include <utility>

#include "svh_internal.h"

namespace svh {

template <typename T> struct CT;
template <> struct CT<double> { typedef double2 t; };
template <> struct CT<float> { typedef float2 t; };

// Store of an intermediate that the next pass streams back in: nontemporal
// (no reuse expected in the caches before then).
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
  typedef float __attribute__((ext_vector_type(2))) f2;
  const f2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<f2*>(p));
}
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  typedef double __attribute__((ext_vector_type(2))) d2;
  const d2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<d2*>(p));
}

// Load of an intermediate that is read once (nontemporal).
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  typedef float __attribute__((ext_vector_type(2))) f2;
  const f2 t = __builtin_nontemporal_load(reinterpret_cast<const f2*>(p));
  return float2{t.x, t.y};
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  typedef double __attribute__((ext_vector_type(2))) d2;
  const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
  return double2{t.x, t.y};
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { return C{a.x * s, a.y * s}; }
// multiply by DIR * i
template <int DIR, typename C> __device__ __forceinline__ C mul_i(C a) {
  return DIR < 0 ? C{a.y, -a.x} : C{-a.y, a.x};
}

template <int DIR, typename C> __device__ __forceinline__ void dft2(C* v) {
  const C a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C& v0, C& v1, C& v2, C& v3) {
  const C a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3);
  const C a3 = mul_i<DIR>(csub(v1, v3));
  v0 = cadd(a0, a2);
  v2 = csub(a0, a2);
  v1 = cadd(a1, a3);
  v3 = csub(a1, a3);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C* v) { dft4<DIR>(v[0], v[1], v[2], v[3]); }

template <int DIR, typename C> __device__ __forceinline__ void dft8(C* v) {
  typedef decltype(v[0].x) T;
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  const T h = (T)0.70710678118654752440;
  // o1 *= w^1, o2 *= w^2 = DIR i, o3 *= w^3 with w = exp(DIR i pi / 4)
  o1 = C{h * (o1.x - DIR * o1.y), h * (o1.y + DIR * o1.x)};
  o2 = mul_i<DIR>(o2);
  o3 = C{h * (-o3.x - DIR * o3.y), h * (-o3.y + DIR * o3.x)};
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <int DIR, typename C> __device__ __forceinline__ void dft3(C* v) {
  typedef decltype(v[0].x) T;
  const T s3 = (T)0.86602540378443864676;
  const C t1 = cadd(v[1], v[2]);
  const C t2 = C{v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y};
  const C d = mul_i<DIR>(cscale(csub(v[1], v[2]), s3));
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, d);
  v[2] = csub(t2, d);
}

template <int R, int DIR, typename C> __device__ __forceinline__ void dft(C* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else dft8<DIR>(v);
}

// Transform of R points (R even) whose upper half, inputs R/2 .. R-1, is zero:
// the first layer of the radix-2 split reduces to copies.
template <int R, int DIR, typename C> __device__ __forceinline__ void dft_lohalf(C* v) {
  static_assert(R % 2 == 0, "even radix");
  if constexpr (R == 2) {
    v[1] = v[0];
  } else if constexpr (R == 4) {
    const C a0 = v[0], a2 = v[1], a3 = mul_i<DIR>(v[1]);
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a0, a3);
    v[3] = csub(a0, a3);
  } else {
    typedef decltype(v[0].x) T;
    // 4-point transforms of (v0, v2, 0, 0) and (v1, v3, 0, 0)
    const C ie = mul_i<DIR>(v[2]), io = mul_i<DIR>(v[3]);
    const C e0 = cadd(v[0], v[2]), e2 = csub(v[0], v[2]), e1 = cadd(v[0], ie), e3 = csub(v[0], ie);
    C o0 = cadd(v[1], v[3]), o2 = csub(v[1], v[3]), o1 = cadd(v[1], io), o3 = csub(v[1], io);
    const T h = (T)0.70710678118654752440;
    o1 = C{h * (o1.x - DIR * o1.y), h * (o1.y + DIR * o1.x)};
    o2 = mul_i<DIR>(o2);
    o3 = C{h * (-o3.x - DIR * o3.y), h * (-o3.y + DIR * o3.x)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
  }
}

template <int R> struct NbMax { static constexpr int v = R == 8 ? 1 : R == 4 ? 2 : R == 3 ? 3 : 4; };

// LDS accessors.  Strided layout: element (n, w) at n * W + w.  Pencil
// layout: element (n, w) at w * Lp + n + n / 8 (one pad slot every eight
// elements keeps the stride-R writes of the first stages off a single bank).
__host__ __device__ constexpr int pencil_pitch(int L) { return L + L / 8 + 1; }
template <typename C, bool STRIDED> struct Lds {
  C* base;
  int W, Lp, w;
  __device__ __forceinline__ C ld(int n) const {
    return STRIDED ? base[n * W + w] : base[w * Lp + n + (n >> 3)];
  }
  __device__ __forceinline__ void st(int n, C v) const {
    if (STRIDED) base[n * W + w] = v;
    else base[w * Lp + n + (n >> 3)] = v;
  }
};

// Global accessors with a split load (kGather: word(), index(), at()) or
// store (kScatter: word(), index(), diag(), put()); the stages issue all
// lookups of a thread before the value accesses.
template <typename C> struct DiagPair { C c, x; };
template <class A, class = void> struct IsGather : std::false_type {};
template <class A> struct IsGather<A, std::void_t<decltype(A::kGather)>> : std::true_type {};
template <class A, class = void> struct IsScatter : std::false_type {};
template <class A> struct IsScatter<A, std::void_t<decltype(A::kScatter)>> : std::true_type {};
// Padding known at compile time.  LowHalf: a transform input whose positions
// at L/2 or beyond are zero (a pencil zero-padded to at least twice its data:
// every even FFT length is at least 2K), read by the first stage only.
// DropUpper: a transform output whose positions at L/2 or beyond are
// discarded (the crop of the inverse), written by the last stage only.
template <class A, class = void> struct LowHalf : std::false_type {};
template <class A> struct LowHalf<A, std::void_t<decltype(A::kLowHalf)>> : std::bool_constant<A::kLowHalf> {};
template <class A, class = void> struct DropUpper : std::false_type {};
template <class A> struct DropUpper<A, std::void_t<decltype(A::kDropUpper)>> : std::bool_constant<A::kDropUpper> {};

// Twiddle table of a length-L transform copied into LDS at `dst` (after the
// block's work area) once per block.  The stages then read twiddles from LDS,
// whose reads are counted apart from the global loads: a stage no longer
// waits for the in-flight loads of the next item when it needs a twiddle
// (vector memory loads complete in issue order).
template <typename C>
__device__ __forceinline__ const C* lds_twiddles(C* dst, const C* __restrict__ tw, int L) {
  for (int i = threadIdx.x; i < L; i += blockDim.x) dst[i] = tw[i];
  __syncthreads();
  return dst;
}
inline size_t twiddle_bytes(int L, size_t csize) { return (size_t)L * csize; }

// Ordering of the LDS accesses of the lanes of one wavefront: the wave's LDS
// instructions execute in program order, so only the compiler must be kept
// from moving accesses across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SYNC_MID: 0 none, 1 block barrier, 2 wavefront ordering (all lanes that
// share the pencil are in one wavefront) between the loads and the stores.
template <typename C, int R, int DIR, int SYNC_MID, class Src, class Dst>
__device__ __forceinline__ void stage_r(int L, int Ns, int j0, int TP, const Src& src, const Dst& dst,
                                        const C* __restrict__ tw) {
  constexpr int NB = NbMax<R>::v;
  constexpr bool SC = IsScatter<Dst>::value;
  // A DropUpper destination takes the last stage (Ns R = L, outputs
  // j + r L/R): with an even radix the outputs r >= R/2 lie at L/2 or beyond,
  // in the discarded padding, so only the first RS outputs of each butterfly
  // are looked up and stored.  A LowHalf source feeds the first stage (Ns = 1,
  // no twiddles): with an even radix its rows r >= R/2 are zero, so only the
  // first RH are read and the butterflies take half their inputs.
  constexpr int RS = (DropUpper<Dst>::value && R % 2 == 0) ? R / 2 : R;
  constexpr int RH = (LowHalf<Src>::value && !IsGather<Src>::value && R % 2 == 0) ? R / 2 : R;
  const int LR = L / R;
  // scatter outputs: indices first, then (after the LDS reads) the operands
  // of the diagonal terms, global loads that overlap the butterflies
  int kk[SC ? NB : 1][SC ? R : 1];
  DiagPair<C> dg[SC ? NB : 1][SC ? R : 1];
  if constexpr (SC) {
    int4 wd[NB][R];
    if constexpr (Dst::kUniform) {
      // last stage (Ns R = L, so base = j) with TP and Ns multiples of 64:
      // the word of j0 + it TP + r Ns is uniform
      const int wq = __builtin_amdgcn_readfirstlane(j0 >> 6);
#pragma unroll
      for (int it = 0; it < NB; ++it)
#pragma unroll
        for (int r = 0; r < RS; ++r) wd[it][r] = dst.row.word_u(wq + ((it * TP + r * Ns) >> 6));
    } else {
#pragma unroll
      for (int it = 0; it < NB; ++it) {
        const int j = j0 + it * TP;
        const int base = (j / Ns) * Ns * R + j % Ns;
#pragma unroll
        for (int r = 0; r < RS; ++r) wd[it][r] = dst.row.word(j < LR ? base + r * Ns : 0);
      }
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int j = j0 + it * TP;
      const int base = (j / Ns) * Ns * R + j % Ns;
#pragma unroll
      for (int r = 0; r < RS; ++r) kk[it][r] = j < LR ? dst.row.index(base + r * Ns, wd[it][r]) : -1;
    }
  }
  C v[NB][R];
  if constexpr (IsGather<Src>::value) {
    // gather source (first stage of a transform): all row words, then all
    // indices, then all value loads
    int4 wg[NB][R];
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int j = j0 + it * TP;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (Src::kUniform)
          wg[it][r] = src.row.word_u(__builtin_amdgcn_readfirstlane(j0 >> 6) + ((it * TP + r * LR) >> 6));
        else
          wg[it][r] = src.row.word(j < LR ? j + r * LR : 0);
      }
    }
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int j = j0 + it * TP;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = src.at(j < LR ? src.row.index(j + r * LR, wg[it][r]) : -1);
    }
  } else {
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int j = j0 + it * TP;
      if (j < LR) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = r < RH ? src.ld(j + r * LR) : C{0, 0};
      }
    }
  }
  if constexpr (SC) {
#pragma unroll
    for (int it = 0; it < NB; ++it)
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        // last stage (n = j + r Ns): outputs r Ns + (it TP ..) wholly past Kx
        // (a uniform branch) are not stored, so they need no operands
        if (Ns * R == L && r * Ns + it * TP >= dst.row.Kx) dg[it][r] = DiagPair<C>{C{0, 0}, C{0, 0}};
        else dg[it][r] = dst.diag(kk[it][r]);
      }
  }
  if constexpr (SYNC_MID == 1) __syncthreads();
  if constexpr (SYNC_MID == 2) wave_sync();
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int j = j0 + it * TP;
    if (j < LR) {
      const int k = j % Ns;
      if (Ns > 1) {
        const int step = L / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C t = tw[r * k * step];
          if (DIR > 0) t.y = -t.y;
          v[it][r] = cmul(v[it][r], t);
        }
      }
      if constexpr (RH < R) dft_lohalf<R, DIR>(v[it]);
      else dft<R, DIR>(v[it]);
      const int base = (j / Ns) * Ns * R + k;
      if constexpr (SC) {
#pragma unroll
        for (int r = 0; r < RS; ++r) dst.put(kk[it][r], v[it][r], dg[it][r]);
      } else {
#pragma unroll
        for (int r = 0; r < RS; ++r) dst.st(base + r * Ns, v[it][r]);
      }
    }
  }
}

template <typename C, int DIR, int SYNC_MID, class Src, class Dst>
__device__ __forceinline__ void stage_any(int R, int L, int Ns, int j0, int TP, const Src& src,
                                          const Dst& dst, const C* tw) {
  switch (R) {
    case 8: stage_r<C, 8, DIR, SYNC_MID>(L, Ns, j0, TP, src, dst, tw); break;
    case 4: stage_r<C, 4, DIR, SYNC_MID>(L, Ns, j0, TP, src, dst, tw); break;
    case 3: stage_r<C, 3, DIR, SYNC_MID>(L, Ns, j0, TP, src, dst, tw); break;
    default: stage_r<C, 2, DIR, SYNC_MID>(L, Ns, j0, TP, src, dst, tw); break;
  }
}

// One full 1D transform of a group of pencils: global -> (LDS stages) -> global.
template <typename C, int DIR, bool STRIDED, class GIn, class GOut>
__device__ __forceinline__ void fft_group(const FftPlan& pl, int j0, const GIn& gin, const GOut& gout,
                                          const Lds<C, STRIDED>& lds, const C* tw) {
  const int L = pl.L, TP = pl.tp;
  if (pl.ns == 1) {
    stage_any<C, DIR, false>(pl.r[0], L, 1, j0, TP, gin, gout, tw);
    return;
  }
  int Ns = 1;
  stage_any<C, DIR, false>(pl.r[0], L, Ns, j0, TP, gin, lds, tw);
  Ns *= pl.r[0];
  __syncthreads();
  for (int s = 1; s < pl.ns - 1; ++s) {
    stage_any<C, DIR, true>(pl.r[s], L, Ns, j0, TP, lds, lds, tw);
    Ns *= pl.r[s];
    __syncthreads();
  }
  stage_any<C, DIR, false>(pl.r[pl.ns - 1], L, Ns, j0, TP, lds, gout, tw);
}

// First stage split into its global loads and the rest (Ns = 1: no twiddles),
// so that a block can issue the loads of its next item before it runs the
// LDS stages of the current one.
template <typename C, int R, class Src>
__device__ __forceinline__ void load0_r(int L, int j0, int TP, const Src& src, C (&v)[12]) {
  constexpr int NB = NbMax<R>::v;
  const int LR = L / R;
  // with an input zero at L/2 and beyond and an even radix, the rows
  // r >= R/2 are zero padding: only the first RH rows are loaded
  constexpr int RH = (LowHalf<Src>::value && R % 2 == 0) ? R / 2 : R;
  if constexpr (IsGather<Src>::value) {
    // all occupancy lookups first, then all value loads
    int4 wd[NB * R];
    if constexpr (Src::kUniform) {
      // TP and LR are multiples of 64: word of j0 + it TP + r LR is uniform
      const int wq = __builtin_amdgcn_readfirstlane(j0 >> 6);
#pragma unroll
      for (int it = 0; it < NB; ++it)
#pragma unroll
        for (int r = 0; r < RH; ++r)
          wd[it * R + r] = r * LR + it * TP >= src.row.Kx ? int4{0, 0, 0, 0}
                                                          : src.row.word_u(wq + ((it * TP + r * LR) >> 6));
    } else {
#pragma unroll
      for (int it = 0; it < NB; ++it) {
        const int j = j0 + it * TP;
#pragma unroll
        for (int r = 0; r < RH; ++r) wd[it * R + r] = src.row.word(j < LR ? j + r * LR : 0);
      }
    }
    int k[NB * R];
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int j = j0 + it * TP;
#pragma unroll
      for (int r = 0; r < RH; ++r) k[it * R + r] = j < LR ? src.row.index(j + r * LR, wd[it * R + r]) : -1;
    }
#pragma unroll
    for (int it = 0; it < NB; ++it)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // rows r LR + (it TP ..) wholly in the zero padding (past Kx on every
        // lane: a uniform branch) load nothing
        if (r >= RH || r * LR + it * TP >= src.row.Kx) v[it * R + r] = C{0, 0};
        else v[it * R + r] = src.at(k[it * R + r]);
      }
  } else {
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int j = j0 + it * TP;
      if (j < LR) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[it * R + r] = r < RH ? src.ld(j + r * LR) : C{0, 0};
      }
    }
  }
}
// LH: the inputs r >= R/2 are zero (the first stage of a LowHalf source, R even).
template <typename C, int R, int DIR, class Dst, bool LH = false>
__device__ __forceinline__ void fin0_r(int L, int j0, int TP, C (&v)[12], const Dst& dst) {
  constexpr int NB = NbMax<R>::v;
  const int LR = L / R;
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int j = j0 + it * TP;
    if (j < LR) {
      if constexpr (LH) dft_lohalf<R, DIR>(&v[it * R]);
      else dft<R, DIR>(&v[it * R]);
#pragma unroll
      for (int r = 0; r < R; ++r) dst.st(j * R + r, v[it * R + r]);
    }
  }
}
template <typename C, class Src>
__device__ __forceinline__ void load0(int R, int L, int j0, int TP, const Src& src, C (&v)[12]) {
  switch (R) {
    case 8: load0_r<C, 8>(L, j0, TP, src, v); break;
    case 4: load0_r<C, 4>(L, j0, TP, src, v); break;
    case 3: load0_r<C, 3>(L, j0, TP, src, v); break;
    default: load0_r<C, 2>(L, j0, TP, src, v); break;
  }
}
template <typename C, int DIR, class Dst>
__device__ __forceinline__ void fin0(int R, int L, int j0, int TP, C (&v)[12], const Dst& dst) {
  switch (R) {
    case 8: fin0_r<C, 8, DIR>(L, j0, TP, v, dst); break;
    case 4: fin0_r<C, 4, DIR>(L, j0, TP, v, dst); break;
    case 3: fin0_r<C, 3, DIR>(L, j0, TP, v, dst); break;
    default: fin0_r<C, 2, DIR>(L, j0, TP, v, dst); break;
  }
}

// First item of a block in the persistent loops.  Blocks are dispatched to
// the 8 XCDs round-robin (block b on XCD b mod 8), each XCD with its own L2;
// when the grid is a multiple of 8, block b starts at item
// (b mod 8) * (grid / 8) + b / 8, so that consecutive items (neighbouring
// column tiles, which share DRAM pages) run on the same XCD.  Each later round
// adds the grid size, so every item is still taken exactly once.
__device__ __forceinline__ int first_item() {
  const int g = gridDim.x, b = blockIdx.x;
  return (g & 7) ? b : (b & 7) * (g >> 3) + (b >> 3);
}

// Persistent loop over items (groups of pencils): item i's first-stage loads
// are issued while item i-1 runs its LDS stages and stores.
template <typename C, int DIR, bool STRIDED, class MkIn, class MkOut>
__device__ __forceinline__ void fft_items(const FftPlan& pl, int j0, int nitems, const MkIn& mk_in,
                                          const MkOut& mk_out, const Lds<C, STRIDED>& lds, const C* tw) {
  const int L = pl.L, TP = pl.tp;
  C v[12];
  int item = first_item();
  if (item < nitems) load0(pl.r[0], L, j0, TP, mk_in(item), v);
  for (; item < nitems; item += gridDim.x) {
    const int next = item + gridDim.x;
    if (pl.ns == 1) {
      fin0<C, DIR>(pl.r[0], L, j0, TP, v, mk_out(item));
      if (next < nitems) load0(pl.r[0], L, j0, TP, mk_in(next), v);
      continue;
    }
    fin0<C, DIR>(pl.r[0], L, j0, TP, v, lds);
    __syncthreads();
    if (next < nitems) load0(pl.r[0], L, j0, TP, mk_in(next), v);
    int Ns = pl.r[0];
    for (int s = 1; s < pl.ns - 1; ++s) {
      stage_any<C, DIR, true>(pl.r[s], L, Ns, j0, TP, lds, lds, tw);
      Ns *= pl.r[s];
      __syncthreads();
    }
    stage_any<C, DIR, false>(pl.r[pl.ns - 1], L, Ns, j0, TP, lds, mk_out(item), tw);
    __syncthreads();
  }
}

// Compile-time plans for the common lengths: all radices, strides and trip
// counts are constants, which keeps every stage in registers (the runtime
// plan above is the fallback for other lengths).
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
template <int R0, int R1 = 1, int R2 = 1, int R3 = 1>
struct PlanC {
  static constexpr bool rt = false;
  static constexpr int ns = R1 == 1 ? 1 : R2 == 1 ? 2 : R3 == 1 ? 3 : 4;
  static constexpr int L = R0 * R1 * R2 * R3;
  static constexpr int r(int s) { return s == 0 ? R0 : s == 1 ? R1 : s == 2 ? R2 : R3; }
  static constexpr int tp = cmin(cmin(L / R0, R1 > 1 ? L / R1 : L), cmin(R2 > 1 ? L / R2 : L, R3 > 1 ? L / R3 : L));
  __host__ __device__ static constexpr int Lof(const FftPlan&) { return L; }
  __host__ __device__ static constexpr int tpof(const FftPlan&) { return tp; }
};
struct PlanRT {
  static constexpr bool rt = true;
  __host__ __device__ static int Lof(const FftPlan& p) { return p.L; }
  __host__ __device__ static int tpof(const FftPlan& p) { return p.tp; }
};

// WAVE: every pencil belongs to one wavefront (its threads and its LDS
// region), so the stages need only the wave's own ordering of its LDS
// accesses instead of block barriers.
template <class P, typename C, int DIR, bool STRIDED, bool WAVE, class MkIn, class MkOut>
__device__ __forceinline__ void fft_items_c(int j0, int nitems, const MkIn& mk_in, const MkOut& mk_out,
                                            const Lds<C, STRIDED>& lds, const C* tw) {
  constexpr int L = P::L, TP = P::tp;
  constexpr int R0 = P::r(0);
  constexpr int SM = WAVE ? 2 : 1;  // in-place stage: wave ordering or block barrier
  auto sync = [] {
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
  };
  // a LowHalf source with an even first radix leaves the upper half of every
  // first-stage butterfly zero (load0_r)
  constexpr bool LH = LowHalf<decltype(mk_in(0))>::value && R0 % 2 == 0;
  C v[12];
  int item = first_item();
  if (item < nitems) load0_r<C, R0>(L, j0, TP, mk_in(item), v);
  for (; item < nitems; item += gridDim.x) {
    const int next = item + gridDim.x;
    if constexpr (P::ns == 1) {
      fin0_r<C, R0, DIR, decltype(mk_out(item)), LH>(L, j0, TP, v, mk_out(item));
      if (next < nitems) load0_r<C, R0>(L, j0, TP, mk_in(next), v);
    } else {
      fin0_r<C, R0, DIR, Lds<C, STRIDED>, LH>(L, j0, TP, v, lds);
      sync();
      if (next < nitems) load0_r<C, R0>(L, j0, TP, mk_in(next), v);
      constexpr int N1 = R0;
      if constexpr (P::ns == 2) {
        stage_r<C, P::r(1), DIR, 0>(L, N1, j0, TP, lds, mk_out(item), tw);
      } else {
        stage_r<C, P::r(1), DIR, SM>(L, N1, j0, TP, lds, lds, tw);
        sync();
        constexpr int N2 = N1 * P::r(1);
        if constexpr (P::ns == 3) {
          stage_r<C, P::r(2), DIR, 0>(L, N2, j0, TP, lds, mk_out(item), tw);
        } else {
          stage_r<C, P::r(2), DIR, SM>(L, N2, j0, TP, lds, lds, tw);
          sync();
          constexpr int N3 = N2 * P::r(2);
          stage_r<C, P::r(3), DIR, 0>(L, N3, j0, TP, lds, mk_out(item), tw);
        }
      }
      sync();
    }
  }
}

template <class P, typename C, int DIR, bool STRIDED, bool WAVE = false, class MkIn, class MkOut>
__device__ __forceinline__ void run_items(const FftPlan& pl, int j0, int nitems, const MkIn& mk_in,
                                          const MkOut& mk_out, const Lds<C, STRIDED>& lds, const C* tw) {
  if constexpr (P::rt) fft_items<C, DIR, STRIDED>(pl, j0, nitems, mk_in, mk_out, lds, tw);
  else fft_items_c<P, C, DIR, STRIDED, WAVE>(j0, nitems, mk_in, mk_out, lds, tw);
}

// Calls f(PlanC<...>{}) for the lengths with a compile-time plan, else f(PlanRT{}).
template <class F>
void with_plan(int L, F&& f) {
  switch (L) {
    case 16: f(PlanC<4, 4>{}); break;
    case 32: f(PlanC<8, 4>{}); break;
    case 64: f(PlanC<8, 8>{}); break;
    case 128: f(PlanC<8, 4, 4>{}); break;
    case 192: f(PlanC<8, 8, 3>{}); break;
    case 256: f(PlanC<8, 8, 4>{}); break;
    case 512: f(PlanC<8, 8, 8>{}); break;
    case 1024: f(PlanC<8, 8, 4, 4>{}); break;
    default: f(PlanRT{}); break;
  }
}

// Block size limit of the pass kernels: 1024 threads for FP32, 512 for FP64
// (which leaves 256 VGPRs per lane for the double-width butterflies).
template <typename T> struct MaxThreads { static constexpr int v = sizeof(T) == 8 ? 512 : 1024; };

// Blocks of a persistent launch: as many as can be resident at once.
inline int persistent_grid(const void* kernel, int threads, size_t shmem, int nitems, int ncu, int mult) {
  if (mult <= 0) return nitems;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, shmem) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const long long g = (long long)per_cu * ncu * mult;
  return (int)(g < nitems ? g : nitems);
}

// Compact index of grid position n from its row's occupancy word (bits low,
// bits high, base, pad), or -1.
__device__ __forceinline__ int xrow_index(int4 wd, int n, bool ok) {
  const unsigned long long bits = ((unsigned long long)(unsigned)wd.y << 32) | (unsigned)wd.x;
  const int b = n & 63;
  // branch-free: all ones when the voxel exists, else zero
  const int sel = -(int)((unsigned)ok & (unsigned)((bits >> b) & 1ull));
  return ((wd.z + __popcll(bits & ((1ull << b) - 1ull))) & sel) | ~sel;
}

// Occupancy words of one grid row.  With UNI, all lanes of a wavefront work
// on the same row (one pencil per wave or more waves per pencil), so a word
// index that is the same on every lane reads through the scalar cache
// (word_u): scalar loads are counted apart from the vector memory accesses,
// and a lookup does not wait for the wave's earlier global loads and stores.
template <bool UNI> struct XRow {
  const XRowWord* __restrict__ xrow;  // all rows (kernel argument)
  int rowoff;                         // first word of this row (wave-uniform with UNI)
  int nw;                             // words per row
  int Kx;
  bool valid;
  __device__ __forceinline__ bool in(int n) const { return valid && n < Kx; }
  // always a valid address (the last word for n >= Kx): an unconditional load
  __device__ __forceinline__ int4 word(int n) const {
    return reinterpret_cast<const int4*>(xrow)[rowoff + ((n < Kx ? n : Kx - 1) >> 6)];
  }
  __device__ __forceinline__ int4 word_u(int wi) const {
    // constant address space: a uniform load there is a scalar load
    typedef __attribute__((address_space(4))) const int cint;
    const cint* q = (const cint*)xrow + 4 * (rowoff + (wi < nw ? wi : nw - 1));
    return int4{q[0], q[1], q[2], q[3]};
  }
  __device__ __forceinline__ int index(int n, int4 wd) const { return xrow_index(wd, n, in(n)); }
};
template <bool UNI>
__device__ __forceinline__ XRow<UNI> make_xrow(const XRowWord* xrow, int row, int nw, int Kx, bool valid) {
  int off = row * nw;
  if constexpr (UNI) off = __builtin_amdgcn_readfirstlane(off);
  return XRow<UNI>{xrow, off, nw, Kx, valid};
}

// Whether a compile-time plan keeps one grid row per wavefront in the x
// passes, with the word index of the first stage's loads and the last stage's
// stores uniform over the wave (threads per pencil and the strides L / r of
// the first and the last stage multiples of 64).
template <class P> constexpr bool uniform_rows() {
  if constexpr (P::rt) return false;
  else return P::tp % 64 == 0 && (P::L / P::r(0)) % 64 == 0 && (P::L / P::r(P::ns - 1)) % 64 == 0;
}

// Whether a compile-time plan runs each pencil of the x passes on exactly one
// wavefront (64 threads per pencil).
template <class P> constexpr bool wave_pencils() {
  if constexpr (P::rt) return false;
  else return P::tp == 64;
}

// Gather accessor of the forward x transform: compact vector -> x pencil.
// Split into the occupancy word load, the index and the value load, so that
// the first stage issues all word loads of a thread, then all value loads
// (ld() does all three for other callers).
template <typename C, bool UNI = false> struct XIn {
  static constexpr bool kGather = true;
  static constexpr bool kLowHalf = true;  // positions >= L/2 >= Kx are padding
  static constexpr bool kUniform = UNI;
  const C* __restrict__ x;              // compact vector of this component
  XRow<UNI> row;
  const C* __restrict__ zero;           // a zero value in device memory
  // empty positions load the zero value: the address is selected, not the
  // value, so the load needs no wait until the value is used
  __device__ __forceinline__ C at(int k) const { return *(k >= 0 ? x + k : zero); }
  __device__ __forceinline__ C ld(int n) const { return at(row.index(n, row.word(n))); }
};
// Scatter accessor of the inverse x transform: scale, diagonal term, compact
// output, split like XIn: a stage looks up all indices of its outputs first.
template <typename C, typename T, bool UNI = false> struct XOut {
  static constexpr bool kScatter = true;
  static constexpr bool kDropUpper = true;  // positions >= L/2 >= Kx are cropped
  static constexpr bool kUniform = UNI;
  C* __restrict__ y;                 // compact output of this component
  const C* __restrict__ x;           // compact input (diagonal term)
  const C* __restrict__ cd;          // c/dx per voxel (nullptr: bare)
  XRow<UNI> row;
  C scale;
  T mass;                            // integral of the squared basis function (eqs. 9, 16-18)
  // operands of the diagonal term, loaded unconditionally (index 0 stands in
  // for empty positions, whose outputs are not stored)
  __device__ __forceinline__ DiagPair<C> diag(int k) const {
    if (!cd) return DiagPair<C>{C{0, 0}, C{0, 0}};
    const int kc = k >= 0 ? k : 0;
    return DiagPair<C>{cd[kc], x[kc]};
  }
  __device__ __forceinline__ void put(int k, C v, const DiagPair<C>& d) const {
    if (k < 0) return;
    C o = cmul(v, scale);
    if (cd) o = cadd(o, cscale(cmul(d.c, d.x), mass));
    y[k] = o;
  }
  __device__ __forceinline__ void st(int n, C v) const {
    const int k = row.index(n, row.word(n));
    put(k, v, diag(k));
  }
};

}  // namespace svh
