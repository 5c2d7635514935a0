// Fused y / z / inverse-y step of the matvec (piecewise-constant basis, direct
// z sum), gfx950.
//
// The separate Y, Z and Yi passes stream the y-padded intermediate (Ly rows
// per plane) through HBM four times.  Here one kernel handles one kx column at
// a time: for every occupied plane it transforms the Ky input rows along y,
// applies the z-space Toeplitz sum over the occupied planes bin by bin, and
// transforms back, keeping y < Ky; only the Ky-row column is read and written.
//
// The column of Ly spectrum bins of all planes does not fit in LDS at once, so
// the bins are taken in r phases (decimation in frequency): phase q holds the
// bins ky = r m + q (m < P = Ly / r), whose values are the length-P transform
// of the folded, twiddled input
//   u_q[n] = sum_t x[n + t P] w^(q (n + t P)),   w = e^(-2 pi i / Ly),
// and whose share of the inverse transform at y = n is w^(-q n) times the
// length-P inverse transform at n mod P.  Each phase adds its share to the
// output column.
//
// Buffers use a transposed layout so that the y columns are contiguous:
// element (vec, plane, kx, y) at (vec * nzp + plane) * pq + kx * cp + y.  The
// x passes of this path store (forward) and load (inverse) through LDS so
// that their global accesses stay contiguous runs of WX rows.
#include "fft_core.h"

namespace svh {

GeoT make_geo_t(const svh_problem* p, size_t cs) {
  GeoT g;
  const int line = (int)(128 / cs);
  g.cp = (p->K[1] + line - 1) / line * line + line;  // whole 128-byte lines, odd line count
  g.pq = (long long)p->L[0] * g.cp + (long long)(256 / cs);
  return g;
}

// Threads per pencil of the compile-time or runtime plan of length L.
int plan_tp(const svh_problem* p, int L) {
  int tp = 0;
  with_plan(L, [&](auto tag) {
    using P = decltype(tag);
    if constexpr (P::rt) {
      FftPlan pl;
      tp = make_plan(L, pl) ? pl.tp : 0;
    } else {
      tp = P::tp;
    }
  });
  (void)p;
  return tp;
}

constexpr int kFusedThreads = 256;
constexpr size_t kFusedLds = 64 * 1024;

size_t fused_lds_bytes(const svh_problem* p, int r, size_t cs, size_t ts) {
  const int Pn = p->L[1] / r;
  const int tp = plan_tp(p, Pn);
  if (tp <= 0 || tp > kFusedThreads) return (size_t)-1;
  const int G = kFusedThreads / tp;
  const int nzp = (int)p->zlist.size();
  const int nzr = (nzp + G - 1) / G * G;
  return (size_t)nzr * pencil_pitch(Pn) * cs + (size_t)p->dzset.size() * Pn * ts;
}

// Smallest phase count r (a divisor of Ly with a supported length Ly / r)
// whose working set fits the LDS budget; 0 if none.
int fused_phases(const svh_problem* p, size_t cs, size_t ts) {
  const int Ly = p->L[1];
  for (int r = 1; r <= Ly; ++r) {
    if (Ly % r) continue;
    const int Pn = Ly / r;
    if (Pn < 2 || !supported_length(Pn)) continue;
    if (fused_lds_bytes(p, r, cs, ts) <= kFusedLds) return r;
  }
  return 0;
}

// ------------------------------------------------------------ accessors ----
template <typename C> struct FoldIn {
  const C* __restrict__ col;  // input column, y contiguous
  const C* __restrict__ twy;  // e^(-2 pi i m / Ly)
  int Ky, Pn, Ly, q;
  bool valid;
  __device__ __forceinline__ C ld(int n) const {
    C s{0, 0};
    if (!valid) return s;
    for (int idx = n; idx < Ky; idx += Pn) {
      C v = col[idx];
      if (q) v = cmul(v, twy[(q * idx) % Ly]);
      s = cadd(s, v);
    }
    return s;
  }
};

// Placeholder accessor for the unused source or destination of fft_batch.
template <typename C> struct NoDst {
  __device__ __forceinline__ C ld(int) const { return C{0, 0}; }
  __device__ __forceinline__ void st(int, C) const {}
};

// Product of the radices of the stages before stage S.
template <class P, int S> struct NsBefore {
  static constexpr int v = S == 0 ? 1 : NsBefore<P, (S > 0 ? S - 1 : 0)>::v * P::r(S > 0 ? S - 1 : 0);
};
template <class P> struct NsBefore<P, 0> { static constexpr int v = 1; };

// One transform of nrd rounds of G pencils (pencil j = rd * G + w, LDS pencil
// layout with pitch PP).  Stage 0 reads mksrc(j) unless FIRST_INPLACE (then
// the pencil itself); the last stage writes mkdst(j) if LAST_TO_DST, else the
// pencil.  WAVE: the TP lanes of a pencil lie in one wavefront (TP divides
// 64), so the stages only need wavefront ordering and one block barrier
// closes the transform; otherwise every stage ends with a block barrier.
template <class P, int S, typename C, int DIR, bool FIRST_INPLACE, bool LAST_TO_DST, bool WAVE, class MkSrc,
          class MkDst>
__device__ __forceinline__ void stages_c(int nrd, int G, int w, int j0, const MkSrc& mksrc, const MkDst& mkdst,
                                         C* work, int PP, const C* tw) {
  if constexpr (S < P::ns) {
    constexpr int Ns = NsBefore<P, S>::v;
    constexpr int R = P::r(S);
    constexpr bool src_lds = !(S == 0 && !FIRST_INPLACE);
    constexpr bool dst_lds = !(S == P::ns - 1 && LAST_TO_DST);
    constexpr int SM = WAVE ? 2 : 1;
    for (int rd = 0; rd < nrd; ++rd) {
      const int j = rd * G + w;
      Lds<C, false> d{work, 0, PP, j};
      if constexpr (src_lds && dst_lds) stage_r<C, R, DIR, SM>(P::L, Ns, j0, P::tp, d, d, tw);
      else if constexpr (src_lds) stage_r<C, R, DIR, 0>(P::L, Ns, j0, P::tp, d, mkdst(j), tw);
      else if constexpr (dst_lds) stage_r<C, R, DIR, 0>(P::L, Ns, j0, P::tp, mksrc(j), d, tw);
      else stage_r<C, R, DIR, 0>(P::L, Ns, j0, P::tp, mksrc(j), mkdst(j), tw);
    }
    if constexpr (WAVE && S + 1 < P::ns) wave_sync();
    else __syncthreads();
    stages_c<P, S + 1, C, DIR, FIRST_INPLACE, LAST_TO_DST, WAVE>(nrd, G, w, j0, mksrc, mkdst, work, PP, tw);
  }
}

template <class P, typename C, int DIR, bool FIRST_INPLACE, bool LAST_TO_DST, class MkSrc, class MkDst>
__device__ __forceinline__ void fft_batch(const FftPlan& pl, int nrd, int G, int w, int j0, const MkSrc& mksrc,
                                          const MkDst& mkdst, C* work, int PP, const C* tw) {
  if constexpr (!P::rt) {
    constexpr bool wave = 64 % P::tp == 0;
    stages_c<P, 0, C, DIR, FIRST_INPLACE, LAST_TO_DST, wave>(nrd, G, w, j0, mksrc, mkdst, work, PP, tw);
  } else {
    const int L = pl.L, TP = pl.tp;
    int Ns = 1;
    for (int s = 0; s < pl.ns; ++s) {
      const bool src_lds = !(s == 0 && !FIRST_INPLACE);
      const bool dst_lds = !(s == pl.ns - 1 && LAST_TO_DST);
      for (int rd = 0; rd < nrd; ++rd) {
        const int j = rd * G + w;
        Lds<C, false> d{work, 0, PP, j};
        if (src_lds && dst_lds) stage_any<C, DIR, 1>(pl.r[s], L, Ns, j0, TP, d, d, tw);
        else if (src_lds) stage_any<C, DIR, 0>(pl.r[s], L, Ns, j0, TP, d, mkdst(j), tw);
        else if (dst_lds) stage_any<C, DIR, 0>(pl.r[s], L, Ns, j0, TP, mksrc(j), d, tw);
        else stage_any<C, DIR, 0>(pl.r[s], L, Ns, j0, TP, mksrc(j), mkdst(j), tw);
      }
      Ns *= pl.r[s];
      __syncthreads();
    }
  }
}

// ----------------------------------------------------- X pass, transposed --
// Item = (vec, plane, group of WX consecutive y rows): gather, forward FFT
// along x in LDS, store column-major (runs of WX rows per kx).
template <typename T, class P>
__global__ void __launch_bounds__(MaxThreads<T>::v) k_pass_xt(FftPlan pl, GeoT gt, int WX, int Kx, int Ky, int nzp, int K,
                                                  int nvec, int ncomp, long long ldx,
                                                  const XRowWord* __restrict__ xrow,
                                                  const typename CT<T>::t* __restrict__ x,
                                                  typename CT<T>::t* __restrict__ At,
                                                  const typename CT<T>::t* __restrict__ tw) {
  typedef typename CT<T>::t C;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x, nt = blockDim.x;
  const int TP = P::tpof(pl), Lx = P::Lof(pl);
  const int PP = pencil_pitch(Lx);
  const int w = t / TP, j0 = t % TP;
  const int ngy = (Ky + WX - 1) / WX;
  const int nitems = nvec * nzp * ngy;
  const int nw = (Kx + 63) >> 6;  // occupancy words per row
  // one pencil (grid row) per wavefront: row words through the scalar cache
  constexpr bool UNI = wave_pencils<P>() && uniform_rows<P>();
  // the word array ends with one zero word, the zero value of empty positions
  const typename CT<T>::t* zero = reinterpret_cast<const typename CT<T>::t*>(xrow + (size_t)nzp * Ky * nw);
  const C* twl = lds_twiddles(lds + (size_t)WX * PP, tw, Lx);
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int gy = item % ngy;
    const int vz = item / ngy;  // vec * nzp + plane
    const int vec = vz / nzp, zp = vz % nzp;
    auto mksrc = [&](int jj) {
      const int y = gy * WX + jj;
      const bool ok = y < Ky;
      return XIn<C, UNI>{x + (size_t)(vec / ncomp) * ldx + (size_t)(vec % ncomp) * K,
                         make_xrow<UNI>(xrow, zp * Ky + (ok ? y : 0), nw, Kx, ok), zero};
    };
    fft_batch<P, C, -1, false, false>(pl, 1, WX, w, j0, mksrc, [](int) { return NoDst<C>{}; }, lds, PP, twl);
    C* col = At + (size_t)vz * gt.pq + gy * WX;
    for (int e = t; e < Lx * WX; e += nt) {
      const int yy = e % WX, kx = e / WX;
      if (gy * WX + yy < Ky) col[(size_t)kx * gt.cp + yy] = lds[yy * PP + kx + (kx >> 3)];
    }
    __syncthreads();
  }
}

// --------------------------------------------- Xi pass, transposed input --
template <typename T, class P>
__global__ void __launch_bounds__(MaxThreads<T>::v) k_pass_xit(FftPlan pl, GeoT gt, int WX, int Kx, int Ky, int nzp, int K,
                                                   int nvec, EpiParams ep, const XRowWord* __restrict__ xrow,
                                                   const typename CT<T>::t* __restrict__ Ot,
                                                   const typename CT<T>::t* __restrict__ x,
                                                   typename CT<T>::t* __restrict__ y,
                                                   const typename CT<T>::t* __restrict__ sconv,
                                                   const typename CT<T>::t* __restrict__ cdiag, T inv_n,
                                                   const typename CT<T>::t* __restrict__ tw) {
  typedef typename CT<T>::t C;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x, nt = blockDim.x;
  const int TP = P::tpof(pl), Lx = P::Lof(pl);
  const int PP = pencil_pitch(Lx);
  const int w = t / TP, j0 = t % TP;
  const int ngy = (Ky + WX - 1) / WX;
  const int nitems = nvec * nzp * ngy;
  const int nw = (Kx + 63) >> 6;  // occupancy words per row
  // one pencil (grid row) per wavefront: row words through the scalar cache
  constexpr bool UNI = wave_pencils<P>() && uniform_rows<P>();
  const C* twl = lds_twiddles(lds + (size_t)WX * PP, tw, Lx);
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int gy = item % ngy;
    const int vz = item / ngy;
    const int vec = vz / nzp, zp = vz % nzp;
    const C* col = Ot + (size_t)vz * gt.pq + gy * WX;
    for (int e = t; e < Lx * WX; e += nt) {
      const int yy = e % WX, kx = e / WX;
      lds[yy * PP + kx + (kx >> 3)] = gy * WX + yy < Ky ? col[(size_t)kx * gt.cp + yy] : C{0, 0};
    }
    __syncthreads();
    const int f = ep.fidx[vec / ep.C];
    const C scale = f >= 0 ? cscale(sconv[f], inv_n) : C{inv_n, 0};
    const C* cd = f >= 0 ? cdiag + (size_t)f * K : nullptr;
    const int rhs = vec / ep.C, comp = vec % ep.C;
    const T mass = comp < 3 ? (T)1 : comp == 3 ? (T)(1.0 / 6.0) : (T)0.5;
    auto mkdst = [&](int jj) {
      const int yy = gy * WX + jj;
      const bool ok = yy < Ky;
      return XOut<C, T, UNI>{y + (size_t)rhs * ep.ldy + (size_t)comp * K, x + (size_t)rhs * ep.ldx + (size_t)comp * K,
                             cd, make_xrow<UNI>(xrow, zp * Ky + (ok ? yy : 0), nw, Kx, ok), scale, mass};
    };
    fft_batch<P, C, +1, true, true>(pl, 1, WX, w, j0, [](int) { return NoDst<C>{}; }, mkdst, lds, PP, twl);
  }
}

// --------------------------------------------------------- fused y/z/yi ----
// Block: one kx column, vectors [v0, v1).  LDS: the phase's spectrum of all
// planes (pencil layout) and the z-space kernel values of the phase's bins.
// qtab: 32 x 32 offset-slot codes (slot of |z_i - z_j| in dzset), four per word.
// Thread t owns rows y = t + 256 b (b < KB) of every plane: it folds them into
// the phase's input and accumulates their share of every phase in registers,
// so each column is read once per phase (from L2 after the first) and written
// once.
template <typename T, class P, int NZ, int KB>
__global__ void __launch_bounds__(256) k_yzy(FftPlan pl, GeoT gt, int Lx, int Ky, int Ly, int r, int nzp, int nd,
                                             int nvec, int vpb, const uint32_t* __restrict__ qtab,
                                             const T* __restrict__ g, const typename CT<T>::t* __restrict__ in,
                                             typename CT<T>::t* __restrict__ out,
                                             const typename CT<T>::t* __restrict__ twp,
                                             const typename CT<T>::t* __restrict__ twy) {
  typedef typename CT<T>::t C;
  extern __shared__ unsigned char smem_raw[];
  const int Pn = P::Lof(pl), TP = P::tpof(pl);
  const int PP = pencil_pitch(Pn);
  const int G = kFusedThreads / TP;
  const int nrd = (nzp + G - 1) / G;
  C* work = reinterpret_cast<C*>(smem_raw);
  T* gs = reinterpret_cast<T*>(work + (size_t)nrd * G * PP);
  const int t = threadIdx.x;
  const int w = t < G * TP ? t / TP : 0;
  const int j0 = t < G * TP ? t % TP : (1 << 20);  // idle threads take no butterfly
  const int kx = blockIdx.x;
  const int v0 = blockIdx.y * vpb, v1 = min(nvec, v0 + vpb);
  const int nfold = (Ky + Pn - 1) / Pn;  // input rows folded onto one bin row
  const int tpb = Pn >= kFusedThreads ? 1 : kFusedThreads / Pn;  // threads per bin in the z sum
  auto nodst = [](int) { return NoDst<C>{}; };
  // padding pencils (transformed along with the planes) stay zero
  for (int e = t; e < (nrd * G - nzp) * Pn; e += kFusedThreads) {
    const int j = nzp + e / Pn, n = e % Pn;
    work[j * PP + n + (n >> 3)] = C{0, 0};
  }
  for (int vec = v0; vec < v1; ++vec) {
    const C* col = in + (size_t)vec * nzp * gt.pq + (size_t)kx * gt.cp;
    C acc[KB][NZ];
    for (int q = 0; q < r; ++q) {
      if (r > 1 || vec == v0) {
        for (int e = t; e < nd * Pn; e += kFusedThreads) {
          const int s = e / Pn, m = e - s * Pn;
          gs[e] = g[((size_t)s * Lx + kx) * Ly + (size_t)r * m + q];
        }
      }
      // fold: work[j][n'] = sum_f x[j][n' + f Pn] w^(q (n' + f Pn)); thread t
      // owns the positions n' = t + 256 k in every pass
      for (int f = 0; f < nfold; ++f) {
        for (int np = t; np < Pn; np += kFusedThreads) {
          const int n = np + f * Pn;
          const bool in_col = n < Ky;
          C tq{1, 0};
          if (q && in_col) tq = twy[(q * n) % Ly];
          C xv[NZ];
#pragma unroll
          for (int j = 0; j < NZ; ++j) xv[j] = (j < nzp && in_col) ? col[(size_t)j * gt.pq + n] : C{0, 0};
          const int o = np + (np >> 3);
#pragma unroll
          for (int j = 0; j < NZ; ++j) {
            if (j >= nzp) continue;
            const C v = q ? cmul(xv[j], tq) : xv[j];
            work[j * PP + o] = f ? cadd(work[j * PP + o], v) : v;
          }
        }
      }
      __syncthreads();
      // forward length-Pn transform of every plane, in place
      fft_batch<P, C, -1, true, false>(pl, nrd, G, w, j0, nodst, nodst, work, PP, twp);
      // z-space Toeplitz sum per bin
      if (tpb == 1) {
        for (int m = t; m < Pn; m += kFusedThreads) {
          const int mo = m + (m >> 3);
          C xin[NZ];
#pragma unroll
          for (int j = 0; j < NZ; ++j) xin[j] = j < nzp ? work[j * PP + mo] : C{0, 0};
          for (int i = 0; i < nzp; ++i) {
            const uint32_t* qrow = qtab + i * 8;
            T ar = 0, ai = 0;
#pragma unroll
            for (int j4 = 0; j4 < NZ / 4; ++j4) {
              const uint32_t c4 = qrow[j4];
#pragma unroll
              for (int bb = 0; bb < 4; ++bb) {
                const T gv = gs[((c4 >> (8 * bb)) & 0x7fu) * Pn + m];
                ar += gv * xin[4 * j4 + bb].x;
                ai += gv * xin[4 * j4 + bb].y;
              }
            }
            work[i * PP + mo] = C{ar, ai};
          }
        }
      } else {
        // tpb threads share bin m and take every tpb-th row; all of them read
        // the bin's inputs before any of them writes a row
        const int nb = Pn * tpb;
        const int m = t % Pn, i0 = t / Pn;
        const int mo = m + (m >> 3);
        C xin[NZ];
        if (t < nb) {
#pragma unroll
          for (int j = 0; j < NZ; ++j) xin[j] = j < nzp ? work[j * PP + mo] : C{0, 0};
        }
        __syncthreads();
        if (t < nb) {
          for (int i = i0; i < nzp; i += tpb) {
            const uint32_t* qrow = qtab + i * 8;
            T ar = 0, ai = 0;
#pragma unroll
            for (int j4 = 0; j4 < NZ / 4; ++j4) {
              const uint32_t c4 = qrow[j4];
#pragma unroll
              for (int bb = 0; bb < 4; ++bb) {
                const T gv = gs[((c4 >> (8 * bb)) & 0x7fu) * Pn + m];
                ar += gv * xin[4 * j4 + bb].x;
                ai += gv * xin[4 * j4 + bb].y;
              }
            }
            work[i * PP + mo] = C{ar, ai};
          }
        }
      }
      __syncthreads();
      // inverse length-Pn transform in place
      fft_batch<P, C, +1, true, false>(pl, nrd, G, w, j0, nodst, nodst, work, PP, twp);
      // this phase's share of the owned rows
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const int n = t + kFusedThreads * b;
        if (n >= Ky) continue;
        const int nm = n % Pn;
        C tq{1, 0};
        if (q) {
          tq = twy[(q * n) % Ly];
          tq.y = -tq.y;
        }
#pragma unroll
        for (int j = 0; j < NZ; ++j) {
          if (j >= nzp) continue;
          const C v = work[j * PP + nm + (nm >> 3)];
          acc[b][j] = q ? cadd(acc[b][j], cmul(v, tq)) : v;
        }
      }
      __syncthreads();
    }
    C* oc = out + (size_t)vec * nzp * gt.pq + (size_t)kx * gt.cp;
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const int n = t + kFusedThreads * b;
      if (n >= Ky) continue;
#pragma unroll
      for (int j = 0; j < NZ; ++j)
        if (j < nzp) oc[(size_t)j * gt.pq + n] = acc[b][j];
    }
  }
}

// ------------------------------------------- fused y/z/yi, resident kernel --
// FP32 variant for 1024-thread blocks with 160 KiB of LDS: one kx column per
// block with the z-space kernel values of all Ly bins resident (loaded once
// per block, stored phase-major: [slot][q][m] for bin ky = r m + q), so only
// the input and output columns of each vector cross HBM, once each.  With
// r <= 2 phases of length Pn >= Ky no two input rows fold onto one bin row.
// The input column stays in registers over the phases (the next vector's
// column is loaded meanwhile); per phase the fold into LDS, the length-Pn
// transforms of all planes, the z sum per bin, the inverse transforms and the
// unfold into register accumulators.
constexpr int kYzy2Threads = 1024;
constexpr size_t kYzy2Lds = 160 * 1024;

size_t yzy2_lds_bytes(const svh_problem* p, int r) {
  const int Ly = p->L[1], Pn = Ly / r;
  return (size_t)p->dzset.size() * Ly * sizeof(float) + p->zlist.size() * (size_t)pencil_pitch(Pn) * sizeof(float2) +
         (size_t)(Pn + Ly) * sizeof(float2);
}

// Phase count for k_yzy2 (0: not applicable): r = Ly / Pn in {1, 2} with Pn
// in {128, 256} (the instantiated transforms), Ky <= Pn, and the working set
// within the LDS.
int yzy2_phases(const svh_problem* p) {
  if (p->C != 3 || p->zlist.size() > (size_t)kMaxDirectPlanes || p->dzset.empty() ||
      p->dzset.size() > (size_t)kMaxDz5)
    return 0;
  const int Ly = p->L[1], Ky = p->K[1];
  for (int r = 1; r <= 2; ++r) {
    if (Ly % r) continue;
    const int Pn = Ly / r;
    if ((Pn != 128 && Pn != 256) || Ky > Pn) continue;
    if (yzy2_lds_bytes(p, r) <= kYzy2Lds) return r;
  }
  return 0;
}

template <class P, int NZ>
__global__ void __launch_bounds__(1024) k_yzy2(GeoT gt, int Lx, int Ky, int Ly, int r, int nzp, int nd, int nvec,
                                               const uint32_t* __restrict__ qtab, const float* __restrict__ g,
                                               const float2* __restrict__ in, float2* __restrict__ out,
                                               const float2* __restrict__ twy) {
  typedef float2 C;
  constexpr int NT = kYzy2Threads;
  constexpr int Pn = P::L, TP = P::tp, PP = pencil_pitch(Pn);
  constexpr int TPB = NT / Pn;                 // threads per bin in the z sum
  constexpr int RS = (NZ + TPB - 1) / TPB;     // rows per thread in the z sum
  constexpr int KM = (NZ * Pn + NT - 1) / NT;  // owned input elements (Ky <= Pn)
  constexpr int NW = (NZ + 3) / 4;             // code words per row
  extern __shared__ unsigned char smem_raw[];
  float* gs = reinterpret_cast<float*>(smem_raw);          // [slot][q][m]
  C* work = reinterpret_cast<C*>(gs + (size_t)nd * Ly);    // [plane][PP]
  C* tpl = work + (size_t)nzp * PP;                        // e^(-2 pi i m / Pn)
  C* tyl = tpl + Pn;                                       // e^(-2 pi i n / Ly)
  const int t = threadIdx.x;
  const int kx = blockIdx.x;
  for (int e = t; e < nd * Ly; e += NT) {
    const int sl = e / Ly, ky = e - sl * Ly;
    gs[(sl * r + ky % r) * Pn + ky / r] = g[((size_t)sl * Lx + kx) * Ly + ky];
  }
  for (int e = t; e < Pn; e += NT) tpl[e] = twy[e * r];
  for (int e = t; e < Ly; e += NT) tyl[e] = twy[e];
  // owned input elements e = t + NT k: plane j = e / Ky, row n = e % Ky
  const int nel = nzp * Ky;
  int jn[KM];  // j << 16 | n, or -1
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const int e = t + NT * k;
    jn[k] = e < nel ? ((e / Ky) << 16) | (e % Ky) : -1;
  }
  // transform roles: pencil w (one plane), lanes of a pencil within a wave
  constexpr int G = NT / TP;
  const int w = t / TP;
  const int j0 = w < nzp ? t % TP : (1 << 20);  // threads of absent planes take no butterfly
  // z-sum roles: bin m, rows i0 + TPB s (i0 is the same on the whole wave);
  // the offset-slot codes of the rows, four per word (zero past nzp)
  const int m = t % Pn;
  const int i0 = __builtin_amdgcn_readfirstlane(t / Pn);
  const int mo = m + (m >> 3);
  auto nodst = [](int) { return NoDst<C>{}; };
  C xn[KM];
  auto fetch = [&](int vec) {
    const C* col = in + (size_t)vec * nzp * gt.pq + (size_t)kx * gt.cp;
#pragma unroll
    for (int k = 0; k < KM; ++k)
      xn[k] = jn[k] >= 0 ? col[(size_t)(jn[k] >> 16) * gt.pq + (jn[k] & 0xffff)] : C{0, 0};
  };
  if (nvec > 0) fetch(0);
  for (int vec = 0; vec < nvec; ++vec) {
    C xc[KM], acc[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      xc[k] = xn[k];
      acc[k] = C{0, 0};
    }
    if (vec + 1 < nvec) fetch(vec + 1);
    for (int q = 0; q < r; ++q) {
      __syncthreads();  // the previous phase is done with work (first pass: tables loaded)
      // fold: work[j][n] = x[j][n] w^(q n) for n < Ky, zero up to Pn
      for (int e = t; e < nzp * (Pn - Ky); e += NT) {
        const int j = e / (Pn - Ky), np = Ky + e % (Pn - Ky);
        work[j * PP + np + (np >> 3)] = C{0, 0};
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (jn[k] < 0) continue;
        const int j = jn[k] >> 16, n = jn[k] & 0xffff;
        work[j * PP + n + (n >> 3)] = q ? cmul(xc[k], tyl[(q * n) % Ly]) : xc[k];
      }
      __syncthreads();
      stages_c<P, 0, C, -1, true, false, true>(1, G, w, j0, nodst, nodst, work, PP, tpl);
      // z sum of bin ky = r m + q: y[i] = sum_j g(slot(i, j)) x[j]
      C yr[RS];
#pragma unroll
      for (int s = 0; s < RS; ++s) yr[s] = C{0, 0};
      const float* gq = gs + (size_t)q * Pn + m;
      const int rPn = r * Pn;
      // planes in groups of four: the rows' code words of the group (scalar
      // loads), then the group's plane values and kernel values (LDS)
#pragma unroll 1
      for (int j4 = 0; j4 < NW; ++j4) {
        uint32_t cw[RS];
#pragma unroll
        for (int s = 0; s < RS; ++s) cw[s] = qtab[(i0 + TPB * s) * 8 + j4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int j = 4 * j4 + b;
          C xj = work[(j < nzp ? j : 0) * PP + mo];
          if (j >= nzp) xj = C{0, 0};
#pragma unroll
          for (int s = 0; s < RS; ++s) {
            const uint32_t code = (cw[s] >> (8 * b)) & 0x7fu;
            const float gv = gq[code * rPn];
            yr[s].x += gv * xj.x;
            yr[s].y += gv * xj.y;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int i = i0 + TPB * s;
        if (i < nzp) work[i * PP + mo] = yr[s];
      }
      __syncthreads();
      stages_c<P, 0, C, +1, true, false, true>(1, G, w, j0, nodst, nodst, work, PP, tpl);
      // unfold: this phase's share w^(-q n) x (length-Pn inverse transform at n)
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (jn[k] < 0) continue;
        const int j = jn[k] >> 16, n = jn[k] & 0xffff;
        C v = work[j * PP + n + (n >> 3)];
        if (q) {
          C tq = tyl[(q * n) % Ly];
          tq.y = -tq.y;
          v = cmul(v, tq);
        }
        acc[k] = cadd(acc[k], v);
      }
    }
    C* oc = out + (size_t)vec * nzp * gt.pq + (size_t)kx * gt.cp;
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (jn[k] >= 0) oc[(size_t)(jn[k] >> 16) * gt.pq + (jn[k] & 0xffff)] = acc[k];
  }
}

// ------------------------------------------------------------ launcher ----
static int rows_per_block_xt(int tp, int Lx, size_t cs) {
  // contiguous runs of 128 bytes when the block (1024 threads FP32, 512 FP64)
  // and its LDS pencils (<= 64 KiB) allow, else 64 bytes, ...
  const int maxt = cs == 16 ? 512 : 1024;
  int WX = (int)(128 / cs);
  while (WX > 1 && (WX * tp > maxt || (size_t)WX * pencil_pitch(Lx) * cs > 65536)) WX /= 2;
  return WX;
}

bool fused_eligible(const svh_problem* p) {
  if (p->C != 3 || p->zlist.size() > (size_t)kMaxDirectPlanes || p->dzset.empty() ||
      p->dzset.size() > (size_t)kMaxDz5)
    return false;
  return p->fused_r[0] > 0 && p->fused_r[1] > 0;
}

bool use_fused(const svh_problem* p, svh_prec prec) {
  if (!fused_eligible(p)) return false;
  if (p->zstep == SVH_ZSTEP_FUSED) return true;
  return p->zstep == SVH_ZSTEP_AUTO && p->auto_fused[prec == SVH_FP64 ? SVH_FP64 : SVH_FP32];
}

template <typename T>
hipError_t launch_matvec_chunk_fused(const svh_problem* p, int nvec, const EpiParams& ep, const void* xv, void* yv,
                                     void* Av, void* Ov, const void* gk, hipStream_t s, hipEvent_t* ev) {
  typedef typename CT<T>::t C;
  const bool dbl = sizeof(T) == 8;
  const C* x = static_cast<const C*>(xv);
  C* y = static_cast<C*>(yv);
  C* At = static_cast<C*>(Av);
  C* Ot = static_cast<C*>(Ov);
  const C* tw[3];
  for (int a = 0; a < 3; ++a)
    tw[a] = dbl ? reinterpret_cast<const C*>(p->d_tw64[a]) : reinterpret_cast<const C*>(p->d_tw32[a]);
  const C* twp = dbl ? reinterpret_cast<const C*>(p->d_twp64) : reinterpret_cast<const C*>(p->d_twp32);
  const int Kx = p->K[0], Ky = p->K[1];
  const int Lx = p->L[0], Ly = p->L[1];
  const int nzp = (int)p->zlist.size();
  const int nd = (int)p->dzset.size();
  const int K = p->nvox;
  const Tune& tn = p->tune[dbl ? SVH_FP64 : SVH_FP32];
  const GeoT gt = make_geo_t(p, sizeof(C));
  const int r = p->fused_r[dbl ? 0 : 1];
  const int Pn = Ly / r;
  if (ev) hipEventRecord(ev[0], s);
  with_plan(Lx, [&](auto tag) {
    using P = decltype(tag);
    const FftPlan& pl = p->plan[0];
    const int tp = P::tpof(pl);
    const int WX = rows_per_block_xt(tp, Lx, sizeof(C));
    const int nitems = nvec * nzp * ((Ky + WX - 1) / WX);
    const size_t sh = (size_t)WX * pencil_pitch(Lx) * sizeof(C) + twiddle_bytes(Lx, sizeof(C));
    const int g = persistent_grid((const void*)k_pass_xt<T, P>, WX * tp, sh, nitems, p->ncu, tn.grid_mult[0]);
    hipLaunchKernelGGL((k_pass_xt<T, P>), dim3(g), dim3(WX * tp), sh, s, pl, gt, WX, Kx, Ky, nzp, K, nvec, ep.C,
                       ep.ldx, p->d_xrow, x, At, tw[0]);
  });
  if (ev) hipEventRecord(ev[1], s);
  if constexpr (sizeof(T) == 4) {
    if (p->fused2_r > 0) {
      const int r2 = p->fused2_r, P2 = Ly / r2;
      const size_t sh = yzy2_lds_bytes(p, r2);
      const uint32_t* qt = reinterpret_cast<const uint32_t*>(p->d_qtab);
      const float* gg = static_cast<const float*>(gk);
      const int NZ = nzp <= 8 ? 8 : nzp <= 16 ? 16 : nzp <= 24 ? 24 : 32;
      with_plan(P2, [&](auto tag) {
        using P = decltype(tag);
        if constexpr (!P::rt) {
          if constexpr (P::L == 128 || P::L == 256) {
            auto go = [&](auto nzt) {
              constexpr int NZc = decltype(nzt)::value;
              auto kern = k_yzy2<P, NZc>;
              hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
              hipLaunchKernelGGL(kern, dim3(Lx), dim3(kYzy2Threads), sh, s, gt, Lx, Ky, Ly, r2, nzp, nd, nvec, qt, gg,
                                 reinterpret_cast<const float2*>(At), reinterpret_cast<float2*>(Ot),
                                 reinterpret_cast<const float2*>(tw[1]));
            };
            switch (NZ) {
              case 8: go(std::integral_constant<int, 8>{}); break;
              case 16: go(std::integral_constant<int, 16>{}); break;
              case 24: go(std::integral_constant<int, 24>{}); break;
              default: go(std::integral_constant<int, 32>{}); break;
            }
          }
        }
      });
    }
  }
  if (sizeof(T) == 8 || p->fused2_r <= 0) {
    FftPlan pp;
    make_plan(Pn, pp);
    with_plan(Pn, [&](auto tag) {
      using P = decltype(tag);
      const int tp = P::rt ? pp.tp : P::tpof(pp);
      const int G = kFusedThreads / tp;
      const int nrd = (nzp + G - 1) / G;
      const size_t sh = (size_t)nrd * G * pencil_pitch(Pn) * sizeof(C) + (size_t)nd * Pn * sizeof(T);
      int vpb = nvec;
      while (vpb > 1 && (long long)Lx * ((nvec + vpb - 1) / vpb) < 2048) vpb = (vpb + 1) / 2;
      dim3 grid(Lx, (nvec + vpb - 1) / vpb);
      const uint32_t* qt = reinterpret_cast<const uint32_t*>(p->d_qtab);
      const T* gg = static_cast<const T*>(gk);
      const int NZ = nzp <= 8 ? 8 : nzp <= 16 ? 16 : nzp <= 24 ? 24 : 32;
      auto go = [&](auto nzt, auto kbt) {
        constexpr int NZc = decltype(nzt)::value, KBc = decltype(kbt)::value;
        hipLaunchKernelGGL((k_yzy<T, P, NZc, KBc>), grid, dim3(kFusedThreads), sh, s, pp, gt, Lx, Ky, Ly, r, nzp, nd,
                           nvec, vpb, qt, gg, At, Ot, twp, tw[1]);
      };
      using K1 = std::integral_constant<int, 1>;
      using K2 = std::integral_constant<int, 2>;
      const bool kb2 = Ky > kFusedThreads;
      switch (NZ) {
        case 8: kb2 ? go(std::integral_constant<int, 8>{}, K2{}) : go(std::integral_constant<int, 8>{}, K1{}); break;
        case 16: kb2 ? go(std::integral_constant<int, 16>{}, K2{}) : go(std::integral_constant<int, 16>{}, K1{}); break;
        case 24: kb2 ? go(std::integral_constant<int, 24>{}, K2{}) : go(std::integral_constant<int, 24>{}, K1{}); break;
        default: kb2 ? go(std::integral_constant<int, 32>{}, K2{}) : go(std::integral_constant<int, 32>{}, K1{}); break;
      }
    });
  }
  if (ev) {
    hipEventRecord(ev[2], s);
    hipEventRecord(ev[3], s);
    hipEventRecord(ev[4], s);
  }
  with_plan(Lx, [&](auto tag) {
    using P = decltype(tag);
    const FftPlan& pl = p->plan[0];
    const int tp = P::tpof(pl);
    const int WX = rows_per_block_xt(tp, Lx, sizeof(C));
    const int nitems = nvec * nzp * ((Ky + WX - 1) / WX);
    const size_t sh = (size_t)WX * pencil_pitch(Lx) * sizeof(C) + twiddle_bytes(Lx, sizeof(C));
    const int g = persistent_grid((const void*)k_pass_xit<T, P>, WX * tp, sh, nitems, p->ncu, tn.grid_mult[3]);
    const T inv_n = (T)(1.0 / ((double)Lx * Ly));
    const C* sc = dbl ? reinterpret_cast<const C*>(p->d_sconv64) : reinterpret_cast<const C*>(p->d_sconv32);
    const C* cd = dbl ? reinterpret_cast<const C*>(p->d_cdiag64) : reinterpret_cast<const C*>(p->d_cdiag32);
    hipLaunchKernelGGL((k_pass_xit<T, P>), dim3(g), dim3(WX * tp), sh, s, pl, gt, WX, Kx, Ky, nzp, K, nvec, ep,
                       p->d_xrow, Ot, x, y, sc, cd, inv_n, tw[0]);
  });
  if (ev) hipEventRecord(ev[5], s);
  return hipGetLastError();
}

template hipError_t launch_matvec_chunk_fused<double>(const svh_problem*, int, const EpiParams&, const void*, void*,
                                                      void*, void*, const void*, hipStream_t, hipEvent_t*);
template hipError_t launch_matvec_chunk_fused<float>(const svh_problem*, int, const EpiParams&, const void*, void*,
                                                     void*, void*, const void*, hipStream_t, hipEvent_t*);

}  // namespace svh
