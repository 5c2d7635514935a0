// Z step by zero-padded FFT along z (eq. 9 literally), for grids whose
// occupied planes are too many for the direct z sum: one block takes W
// adjacent kx columns of one ky row (W pencils along z) and runs them through
// every item of its share of the batch, so the spectrum values of its pencils
// are read from HBM once per launch.
//
// Per item the occupied planes of the x/y-transformed data are loaded into
// LDS pencils indexed by z (coalesced runs of W x-adjacent values; a pencil's
// threads are consecutive, so the stages of a pencil that fits in one
// wavefront are ordered without block barriers); the first
// forward stage reads the unoccupied positions as zeros, so nothing is
// cleared.  The last forward stage, the spectrum product and the first
// inverse stage run in registers (Stockham: the last forward stage leaves
// bin j + r L/R in the thread that starts the inverse butterfly of the same
// bins).  After the inverse stages only the occupied planes are stored.
//
//  * NC = 1 (three components): an item is one component vector; the
//    product is the real M0 spectrum.
//  * NC = 5 (piecewise-linear basis): an item is one right-hand side of five
//    component vectors coupled by the 17 blocks of eq. 8, written with the
//    seven family spectra S_f (real; the spectrum of the family is j S_f for
//    M1x, M1y, M1z, which are odd along one axis) and u = I2D + I3D,
//    w = I2D - I3D:
//      y_x  = S0 Ix + j S1x u
//      y_y  = S0 Iy - j S1y w
//      y_z  = S0 Iz - 2 j S1z I3D
//      y_2D = j (S1y Iy - S1x Ix) + S2x u + S2y w
//      y_3D = -j (S1x Ix + S1y Iy) + 2 j S1z Iz + S2x u - S2y w + 4 S2z I3D
//    The five components' last-stage values are held in registers while one
//    LDS array is reused for each component's stages.
//
// Spectra are stored folded: S_f at 0 <= k_a <= L_a / 2 per axis, the rest
// by symmetry (S(L - k) = S(k), or -S(k) along the odd axis of an M1 family),
// one eighth of the full grid.  The inverse transform's 1/Lz is folded into
// the product.
#include "fft_core.h"

namespace svh {

namespace {

// LDS pencils in the pencil layout of Lds<C, false> (element (n, w) at
// w * Lp + n + n / 8); positions whose z plane is empty read as zero, and
// so do all positions at Lz/2 or beyond (Lz >= 2 Kz), which the first stage
// does not read.
template <typename C> struct LdsOcc {
  static constexpr bool kLowHalf = true;
  C* base;
  int Lp, w;
  const uint8_t* occ;
  __device__ __forceinline__ C ld(int n) const { return occ[n] ? base[w * Lp + n + (n >> 3)] : C{0, 0}; }
};
__device__ __forceinline__ int pencil_at(int w, int n, int Lp) { return w * Lp + n + (n >> 3); }
// The same pencils as the destination of the last inverse stage: only planes
// below Kz <= Lz/2 are stored afterwards, so outputs at Lz/2 or beyond are
// not written.
template <typename C> struct LdsCrop : Lds<C, false> {
  static constexpr bool kDropUpper = true;
};

// Ordering of the LDS stages of one pencil: the lanes of a pencil are
// consecutive threads, so when the pencils do not straddle wavefronts
// (threads per pencil divide 64) wavefront ordering suffices.
template <bool WAVE> __device__ __forceinline__ void pencil_sync() {
  if constexpr (WAVE) wave_sync();
  else __syncthreads();
}

__device__ __forceinline__ int fold_index(int k, int L) { return k <= L / 2 ? k : L - k; }

// Parity of the seven families along x, y, z (M1 of axis a is odd along a).
__device__ __forceinline__ bool fam_odd(int f, int a) { return f >= 1 && f <= 3 && f - 1 == a; }

// Spectrum value of family f at (kx, ky, kz) from the folded table, times s.
template <typename T>
__device__ __forceinline__ T spec_at(const T* __restrict__ spec, int f, int kx, int ky, int kz, int Lx, int Ly,
                                     int Lz, T s) {
  const int hx = Lx / 2 + 1, hy = Ly / 2 + 1, hz = Lz / 2 + 1;
  const int fx = fold_index(kx, Lx), fy = fold_index(ky, Ly), fz = fold_index(kz, Lz);
  if ((fam_odd(f, 0) && kx > Lx / 2) != (fam_odd(f, 1) && ky > Ly / 2) != (fam_odd(f, 2) && kz > Lz / 2)) s = -s;
  return s * spec[(((size_t)f * hz + fz) * hy + fy) * hx + fx];
}

// Last forward stage (Ns = L/R) of one pencil group: bins j + r L/R of the
// butterflies j = j0 + it TP, into registers.
template <typename C, int R, class Src>
__device__ __forceinline__ void last_forward(int L, int j0, int TP, const Src& src, const C* __restrict__ tw,
                                             C (&v)[12]) {
  constexpr int NB = NbMax<R>::v;
  const int LR = L / R;
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int j = j0 + it * TP;
    if (j < LR) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[it * R + r] = src.ld(j + r * LR);
    }
  }
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int j = j0 + it * TP;
    if (j < LR) {
      if (LR > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[it * R + r] = cmul(v[it * R + r], tw[r * j]);
      }
      dft<R, -1>(&v[it * R]);
    }
  }
}

// First inverse stage (Ns = 1, radix R) from registers holding bins
// j + r L/R: outputs j R + r into the LDS pencils.
template <typename C, int R, class Dst>
__device__ __forceinline__ void first_inverse(int L, int j0, int TP, C (&v)[12], const Dst& dst) {
  constexpr int NB = NbMax<R>::v;
  const int LR = L / R;
#pragma unroll
  for (int it = 0; it < NB; ++it) {
    const int j = j0 + it * TP;
    if (j < LR) {
      dft<R, +1>(&v[it * R]);
#pragma unroll
      for (int r = 0; r < R; ++r) dst.st(j * R + r, v[it * R + r]);
    }
  }
}

template <typename T> struct ZfftArgs {
  typedef typename CT<T>::t C;
  FftPlan pl, ipl;
  Geo geo;
  int W, Lx, Ly, Lz, nzp, nitem, ipb;
  const int32_t* zlist;  // occupied planes
  const T* spec;         // folded spectra [f][kz][ky][kx]
  C* B;                  // [vec][plane slot][ky][kx]
  const C* tw;           // z twiddles, length Lz
};

template <typename T, int NC, int R, bool WAVE>
__device__ __forceinline__ void zfft_items(const ZfftArgs<T>& a, int kx0, int ky, typename CT<T>::t* buf,
                                           const typename CT<T>::t* twl, const int* zl, const uint8_t* occ,
                                           const T* lspec) {
  typedef typename CT<T>::t C;
  constexpr int NB = NbMax<R>::v;
  constexpr int SM = WAVE ? 2 : 1;  // ordering inside a stage
  const int t = threadIdx.x;
  const int W = a.W;
  const int L = a.Lz, TP = a.pl.tp, LR = L / R;
  const int w = t / TP, j0 = t % TP;  // a pencil's lanes are consecutive threads
  const int Lp = pencil_pitch(L);
  const int ns = a.pl.ns;
  const int nthreads = blockDim.x;
  const size_t plane = (size_t)a.geo.pb;
  const int kx = kx0 + w;
  Lds<C, false> lds{buf, W, Lp, w};
  LdsOcc<C> lin{buf, Lp, w, occ};
  // spectrum values of this thread's bins (NC = 1)
  T zv[12];
  if constexpr (NC == 1) {
    const T s = (T)1 / (T)L;
#pragma unroll
    for (int it = 0; it < NB; ++it)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = j0 + it * TP;
        zv[it * R + r] = (j < LR && kx < a.Lx) ? spec_at(a.spec, 0, kx, ky, j + r * LR, a.Lx, a.Ly, L, s) : (T)0;
      }
  }
  const int v0 = blockIdx.y * a.ipb;
  const int v1 = min(a.nitem, v0 + a.ipb);
  // the planes of the next component vector are loaded into registers while
  // the current one runs its stages (the first kPre elements of each thread;
  // longer columns load the rest when they are staged)
  constexpr int kPre = 8;
  const int ne = a.nzp * W;
  C pre[kPre];
  auto col = [&](int vec) { return a.B + (size_t)vec * a.nzp * plane + (size_t)ky * a.geo.rp + kx0; };
  auto fetch = [&](int vec) {
    const C* src = col(vec);
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int e = t + q * nthreads;
      const int sl = e / W, ww = e % W;
      pre[q] = (e < ne && kx0 + ww < a.Lx) ? ld_stream(src + (size_t)sl * plane + ww) : C{0, 0};
    }
  };
  if (v0 < v1) fetch(v0 * NC);
  for (int item = v0; item < v1; ++item) {
    C V[NC][12];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int vec = item * NC + c;
      __syncthreads();  // the previous user of buf is done
#pragma unroll
      for (int q = 0; q < kPre; ++q) {
        const int e = t + q * nthreads;
        const int sl = e / W, ww = e % W;
        if (e < ne && kx0 + ww < a.Lx) buf[pencil_at(ww, zl[sl], Lp)] = pre[q];
      }
      for (int e = t + kPre * nthreads; e < ne; e += nthreads) {
        const int sl = e / W, ww = e % W;
        if (kx0 + ww < a.Lx) buf[pencil_at(ww, zl[sl], Lp)] = ld_stream(col(vec) + (size_t)sl * plane + ww);
      }
      __syncthreads();
      if (vec + 1 < v1 * NC) fetch(vec + 1);
      if (ns == 1) {
        last_forward<C, R>(L, j0, TP, lin, twl, V[c]);
      } else {
        int Ns = 1;
        stage_any<C, -1, SM>(a.pl.r[0], L, Ns, j0, TP, lin, lds, twl);
        Ns *= a.pl.r[0];
        pencil_sync<WAVE>();
        for (int s = 1; s < ns - 1; ++s) {
          stage_any<C, -1, SM>(a.pl.r[s], L, Ns, j0, TP, lds, lds, twl);
          Ns *= a.pl.r[s];
          pencil_sync<WAVE>();
        }
        last_forward<C, R>(L, j0, TP, lds, twl, V[c]);
      }
    }
    // spectrum product, bin by bin
#pragma unroll
    for (int it = 0; it < NB; ++it) {
      const int j = j0 + it * TP;
      if (j >= LR) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = it * R + r;
        if constexpr (NC == 1) {
          V[0][q] = cscale(V[0][q], zv[q]);
        } else {
          const T* sp = lspec + (size_t)(j + r * LR) * W + w;  // [7][L][W]
          const size_t fs = (size_t)L * W;
          const T s0 = sp[0], s1x = sp[fs], s1y = sp[2 * fs], s1z = sp[3 * fs];
          const T s2x = sp[4 * fs], s2y = sp[5 * fs], s2z = sp[6 * fs];
          const C Ix = V[0][q], Iy = V[1][q], Iz = V[2][q], I2 = V[3][q], I3 = V[4][q];
          const C u = cadd(I2, I3), wv = csub(I2, I3);
          // j (a + i b) = (-b + i a)
          auto jm = [](C z, T s) { return C{-s * z.y, s * z.x}; };
          V[0][q] = cadd(cscale(Ix, s0), jm(u, s1x));
          V[1][q] = csub(cscale(Iy, s0), jm(wv, s1y));
          V[2][q] = csub(cscale(Iz, s0), jm(I3, (T)2 * s1z));
          const C m1 = csub(cscale(Iy, s1y), cscale(Ix, s1x));
          V[3][q] = cadd(jm(m1, (T)1), cadd(cscale(u, s2x), cscale(wv, s2y)));
          const C m2 = cadd(cscale(Ix, s1x), cscale(Iy, s1y));
          V[4][q] = cadd(csub(jm(Iz, (T)2 * s1z), jm(m2, (T)1)),
                         cadd(csub(cscale(u, s2x), cscale(wv, s2y)), cscale(I3, (T)4 * s2z)));
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      __syncthreads();  // every thread has read buf (last forward stage / previous store)
      first_inverse<C, R>(L, j0, TP, V[c], lds);
      pencil_sync<WAVE>();
      int Ns = R;
      for (int s = 1; s < ns; ++s) {
        if (s < ns - 1) stage_any<C, +1, SM>(a.ipl.r[s], L, Ns, j0, TP, lds, lds, twl);
        else stage_any<C, +1, SM>(a.ipl.r[s], L, Ns, j0, TP, lds, LdsCrop<C>{lds}, twl);
        Ns *= a.ipl.r[s];
        pencil_sync<WAVE>();
      }
      __syncthreads();  // every pencil's stages are done before the coalesced store
      C* dst = a.B + ((size_t)(item * NC + c) * a.nzp) * plane + (size_t)ky * a.geo.rp + kx0;
      for (int e = t; e < a.nzp * W; e += nthreads) {
        const int sl = e / W, ww = e % W;
        if (kx0 + ww < a.Lx) st_stream(dst + (size_t)sl * plane + ww, buf[pencil_at(ww, zl[sl], Lp)]);
      }
    }
  }
}

}  // namespace

template <typename T, int NC, int R, bool WAVE>
__global__ void __launch_bounds__(256) k_zfft(ZfftArgs<T> a) {
  typedef typename CT<T>::t C;
  extern __shared__ unsigned char smem_raw[];
  const int W = a.W, L = a.Lz;
  C* buf = reinterpret_cast<C*>(smem_raw);               // W pencils of pitch Lp
  C* twd = buf + (size_t)W * pencil_pitch(L);            // [L]
  T* lspec = reinterpret_cast<T*>(twd + L);              // NC = 5: [7][L][W]
  int* zl = reinterpret_cast<int*>(lspec + (NC == 5 ? (size_t)kNFam * L * W : 0));  // [nzp]
  uint8_t* occ = reinterpret_cast<uint8_t*>(zl + a.nzp);  // [L]
  const int t = threadIdx.x;
  const int ntile = (a.Lx + W - 1) / W;
  const int bid = first_item();  // XCD-aware order of the (tile, ky) blocks
  const int tile = bid % ntile, ky = bid / ntile;
  const int kx0 = tile * W;
  for (int i = t; i < L; i += blockDim.x) occ[i] = 0;
  __syncthreads();
  for (int i = t; i < a.nzp; i += blockDim.x) {
    zl[i] = a.zlist[i];
    occ[a.zlist[i]] = 1;
  }
  if constexpr (NC == 5) {
    const T s = (T)1 / (T)L;
    for (int e = t; e < kNFam * L * W; e += blockDim.x) {
      const int w = e % W, n = (e / W) % L, f = e / (W * L);
      const int kx = kx0 + w;
      lspec[e] = kx < a.Lx ? spec_at(a.spec, f, kx, ky, n, a.Lx, a.Ly, L, s) : (T)0;
    }
  }
  const C* twl = lds_twiddles(twd, a.tw, L);  // synchronises
  zfft_items<T, NC, R, WAVE>(a, kx0, ky, buf, twl, zl, occ, lspec);
}

// Pencils per block: 16 (FP32) or 8 (FP64) x-adjacent columns, fewer when
// the threads (W x threads per pencil) would exceed 256.
static int zfft_width(const FftPlan& pl, size_t cs) {
  int W = cs == 8 ? 16 : 8;
  while (W > 1 && W * pl.tp > 256) W /= 2;
  return W;
}

size_t zfft_lds_bytes(const svh_problem* p, size_t cs, int nc) {
  const FftPlan& pl = p->plan[2];
  const int W = zfft_width(pl, cs);
  const size_t ts = cs / 2;
  return (size_t)W * pencil_pitch(pl.L) * cs + (size_t)pl.L * cs + (nc == 5 ? (size_t)kNFam * pl.L * W * ts : 0) +
         p->zlist.size() * sizeof(int) + (size_t)pl.L;
}

template <typename T>
hipError_t launch_zfft(const svh_problem* p, int nvec, void* Bv, const void* spec, hipStream_t s) {
  typedef typename CT<T>::t C;
  ZfftArgs<T> a;
  a.pl = p->plan[2];
  a.ipl = reversed(a.pl);
  a.geo = make_geo(p, sizeof(C));
  a.W = zfft_width(a.pl, sizeof(C));
  a.Lx = p->L[0];
  a.Ly = p->L[1];
  a.Lz = p->L[2];
  a.nzp = (int)p->zlist.size();
  const int nc = p->C == 5 ? 5 : 1;
  a.nitem = nvec / nc;
  a.zlist = p->d_zlist;
  a.spec = static_cast<const T*>(spec);
  a.B = static_cast<C*>(Bv);
  a.tw = reinterpret_cast<const C*>(sizeof(T) == 8 ? (const void*)p->d_tw64[2] : (const void*)p->d_tw32[2]);
  const int ntile = (a.Lx + a.W - 1) / a.W;
  const int nblk = ntile * a.Ly;
  // items per block: all of them unless that leaves fewer than 2048 blocks
  int ipb = a.nitem;
  while (ipb > 1 && (long long)nblk * ((a.nitem + ipb - 1) / ipb) < 2048) ipb = (ipb + 1) / 2;
  a.ipb = ipb;
  dim3 grid(nblk, (a.nitem + ipb - 1) / ipb);
  const size_t sh = zfft_lds_bytes(p, sizeof(C), nc);
  if (sh > (size_t)p->max_lds) return hipErrorInvalidConfiguration;
  const int nt = a.W * a.pl.tp;
  // one kernel per (components, last radix, pencil ordering), so each gets
  // its own register allocation
  const bool wave = 64 % a.pl.tp == 0;
  auto go = [&](auto nct, auto rt, auto wt) {
    constexpr int NCc = decltype(nct)::value, Rc = decltype(rt)::value;
    constexpr bool Wc = decltype(wt)::value;
    hipLaunchKernelGGL((k_zfft<T, NCc, Rc, Wc>), grid, dim3(nt), sh, s, a);
  };
  auto by_r = [&](auto nct, auto wt) {
    switch (a.pl.r[a.pl.ns - 1]) {
      case 8: go(nct, std::integral_constant<int, 8>{}, wt); break;
      case 4: go(nct, std::integral_constant<int, 4>{}, wt); break;
      case 3: go(nct, std::integral_constant<int, 3>{}, wt); break;
      default: go(nct, std::integral_constant<int, 2>{}, wt); break;
    }
  };
  using N1 = std::integral_constant<int, 1>;
  using N5 = std::integral_constant<int, 5>;
  using WT = std::integral_constant<bool, true>;
  using WF = std::integral_constant<bool, false>;
  if (nc == 5) {
    if (wave) by_r(N5{}, WT{});
    else by_r(N5{}, WF{});
  } else {
    if (wave) by_r(N1{}, WT{});
    else by_r(N1{}, WF{});
  }
  return hipGetLastError();
}

template hipError_t launch_zfft<double>(const svh_problem*, int, void*, const void*, hipStream_t);
template hipError_t launch_zfft<float>(const svh_problem*, int, void*, const void*, hipStream_t);

}  // namespace svh
