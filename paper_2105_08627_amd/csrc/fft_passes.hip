// FFT convolution passes of the VIE matrix-vector product (eq. 9), gfx950.
//
// y = s * IFFT3( Zhat .* FFT3( pad(x) ) )[crop] / (Lx Ly Lz) + (c/dx) x
//
// The 3D transforms run as five HBM passes over pencils, each a batched 1D
// mixed-radix Stockham FFT staged through LDS:
//   X  : gather compact x into zero-padded x-pencils, forward FFT along x
//   Y  : forward FFT along y (input half is zero: only y < Ky is read)
//   Z  : forward FFT along z, multiply by the real spectrum, inverse FFT
//        along z, all in one kernel (the last forward and the first inverse
//        butterfly stage share registers)
//   Yi : inverse FFT along y, keep y < Ky
//   Xi : inverse FFT along x, keep x < Kx, scale, add the diagonal term and
//        scatter to the compact output
// Only z planes that hold at least one non-empty voxel are stored between
// passes (the others are zero on input and not needed on output).
#include "fft_core.h"

namespace svh {

// ----------------------------------------------------------------- X pass --
template <typename C> struct RowOut {
  C* __restrict__ row;
  int lim;
  bool valid;
  __device__ __forceinline__ void st(int n, C v) const {
    if (valid && n < lim) st_stream(row + n, v);
  }
};

template <typename T, class P>
__global__ void __launch_bounds__(256) k_pass_x(FftPlan pl, Geo geo, int WX, int Kx, int Ky, int nzp, int K, int nvec,
                                                int ncomp, long long ldx,
                                                 const XRowWord* __restrict__ xrow,
                                                 const typename CT<T>::t* __restrict__ x,
                                                 typename CT<T>::t* __restrict__ A,
                                                 const typename CT<T>::t* __restrict__ tw) {
  typedef typename CT<T>::t C;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x;
  const int TPP = P::tpof(pl);
  const int j0 = t % TPP, w = t / TPP;
  const int NP = nzp * Ky;
  const int ngrp = (NP + WX - 1) / WX;
  const int Lx = P::Lof(pl);
  const int nw = (Kx + 63) >> 6;  // occupancy words per row
  // the word array ends with one zero word, the zero value of empty positions
  const typename CT<T>::t* zero = reinterpret_cast<const typename CT<T>::t*>(xrow + (size_t)nzp * Ky * nw);
  // item = vec * ngrp + pencil group
  auto where = [&](int item, int& vec, int& y, int& zp, bool& valid) {
    vec = item / ngrp;
    const int pen = (item % ngrp) * WX + w;
    valid = pen < NP;
    const int pc = valid ? pen : 0;
    y = pc % Ky;
    zp = pc / Ky;
  };
  auto mk_in = [&](int item) {
    int vec, y, zp;
    bool valid;
    where(item, vec, y, zp, valid);
    return XIn<C, uniform_rows<P>()>{x + (size_t)(vec / ncomp) * ldx + (size_t)(vec % ncomp) * K,
                                     make_xrow<uniform_rows<P>()>(xrow, zp * Ky + y, nw, Kx, valid), zero};
  };
  auto mk_out = [&](int item) {
    int vec, y, zp;
    bool valid;
    where(item, vec, y, zp, valid);
    return RowOut<C>{A + ((size_t)vec * nzp + zp) * geo.pa + (size_t)y * geo.rp, Lx, valid};
  };
  Lds<C, false> acc{lds, WX, pencil_pitch(Lx), w};
  const C* twl = lds_twiddles(lds + (size_t)WX * pencil_pitch(Lx), tw, Lx);
  run_items<P, C, -1, false, wave_pencils<P>()>(pl, j0, ngrp * nvec, mk_in, mk_out, acc, twl);
}

// ------------------------------------------------------------ Y passes ----
template <typename C> struct ColIn {
  const C* __restrict__ base;  // plane start + kx
  int stride, lim;
  bool valid;
  __device__ __forceinline__ C ld(int n) const {
    return (valid && n < lim) ? ld_stream(base + (size_t)n * stride) : C{0, 0};
  }
};
template <typename C> struct ColOut {
  C* __restrict__ base;
  int stride, lim;
  bool valid;
  __device__ __forceinline__ void st(int n, C v) const {
    if (valid && n < lim) st_stream(base + (size_t)n * stride, v);
  }
};

// DIR = -1: A[vec][zp][y < Ky][kx] -> B[vec][zp][ky < Ly][kx]
// DIR = +1: B -> A (crop to y < Ky)
template <typename T, int DIR, class P>
__global__ void __launch_bounds__(MaxThreads<T>::v) k_pass_y(FftPlan pl, Geo geo, int W, int Lx, int Ky, int nzp, int nvec,
                                                 const typename CT<T>::t* __restrict__ in,
                                                 typename CT<T>::t* __restrict__ out,
                                                 const typename CT<T>::t* __restrict__ tw) {
  typedef typename CT<T>::t C;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x;
  const int w = t % W, j0 = t / W;
  const int ntile = (Lx + W - 1) / W;
  const int Ly = P::Lof(pl);
  const int rows_in = DIR < 0 ? Ky : Ly;
  const int rows_out = DIR < 0 ? Ly : Ky;
  // item = (vec * nzp + zp) * ntile + tile
  auto col = [&](int item, bool& valid) {
    const int tile = item % ntile;
    const int vz = item / ntile;  // vec * nzp + zp
    const int kx = tile * W + w;
    valid = kx < Lx;
    return std::make_pair((size_t)vz, valid ? kx : 0);
  };
  auto mk_in = [&](int item) {
    bool valid;
    const auto c = col(item, valid);
    return ColIn<C>{in + c.first * (DIR < 0 ? geo.pa : geo.pb) + c.second, geo.rp, rows_in, valid};
  };
  auto mk_out = [&](int item) {
    bool valid;
    const auto c = col(item, valid);
    return ColOut<C>{out + c.first * (DIR < 0 ? geo.pb : geo.pa) + c.second, geo.rp, rows_out, valid};
  };
  Lds<C, true> acc{lds, W, 0, w};
  const C* twl = lds_twiddles(lds + (size_t)W * Ly, tw, Ly);
  run_items<P, C, DIR, true>(pl, j0, ntile * nzp * nvec, mk_in, mk_out, acc, twl);
}

// ------------------------------------------------- Z step, direct sum ----
// The z-direction product of eq. 9 written in z space: after the x and y
// transforms, pencil (kx, ky) needs y[z_i] = sum_j g(kx, ky, |z_i - z_j|) x[z_j]
// over the occupied planes only, where g is the inverse z transform of the
// circulant spectrum (real and even in the offset because the spectrum is
// real and even).  Exact for any plane set; used when few planes are occupied
// (the padded z FFT then spends almost all of its work on zeros).
// Block: W adjacent kx of one ky, RG row groups (W * RG = NT threads).
// g rows: plane offsets dz < Kz, or (qslot given) the distinct offsets only.
// Thread (w, rg) keeps rows rg, rg + RG, ... of its pencil's nzp x nzp matrix
// in registers for all vectors; each chunk of V vectors is staged through
// LDS with 128/256-byte coalesced loads and updated in place.
template <typename T, int NZ, int RG, int V, int NT>
__global__ void __launch_bounds__(NT) k_zdirect(Geo geo, int Lx, int Ly, int nzp, int nvec, int vpb,
                                                 const int32_t* __restrict__ zlist,
                                                 const uint8_t* __restrict__ qslot,
                                                 const T* __restrict__ g,
                                                 typename CT<T>::t* __restrict__ B) {
  typedef typename CT<T>::t C;
  constexpr int W = NT / RG;
  constexpr int R = (NZ + RG - 1) / RG;
  extern __shared__ unsigned char smem_raw[];
  C* xs = reinterpret_cast<C*>(smem_raw);                    // [V][NZ][W]
  int* zl = reinterpret_cast<int*>(xs + (size_t)V * NZ * W); // [NZ]
  const int t = threadIdx.x;
  const int ntile = (Lx + W - 1) / W;
  const int bid = first_item();  // XCD-aware order of the (tile, ky) blocks
  const int tile = bid % ntile, ky = bid / ntile;
  const int kx0 = tile * W;
  uint8_t* qs = reinterpret_cast<uint8_t*>(zl + NZ);       // [NZ][NZ] slot codes (qslot given)
  for (int i = t; i < NZ; i += NT) zl[i] = i < nzp ? zlist[i] : 0;
  if (qslot)
    for (int e = t; e < NZ * NZ; e += NT) qs[e] = qslot[(e / NZ) * 32 + e % NZ];
  __syncthreads();
  const int w = t % W, rg = t / W;
  const int kx = kx0 + w;
  const bool valid = kx < Lx;
  // rows of this pencil's z matrix, read once per block (x-adjacent lanes)
  T m[R][NZ];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = rg + r * RG;
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      // row of g: the plane offset |z_i - z_j|, or its slot among the
      // distinct offsets when g holds only those (qslot, 32 x 32 codes)
      int d = zl[i < NZ ? i : 0] - zl[j];
      d = d < 0 ? -d : d;
      if (qslot && i < nzp && j < nzp) d = qs[i * NZ + j] & 0x7f;
      m[r][j] = (valid && i < nzp && j < nzp) ? g[((size_t)d * Ly + ky) * Lx + kx] : (T)0;
    }
  }
  const size_t plane = (size_t)geo.pb;
  C* base = B + (size_t)ky * geo.rp + kx0;
  const int vbeg = blockIdx.y * vpb;
  const int vend = min(nvec, vbeg + vpb);
  // staged element e of a chunk: ww = e % W, j = (e / W) % NZ, v = e / (W NZ);
  // thread t stages e = t + NT q, q < EPT
  constexpr int EPT = (V * NZ * W + NT - 1) / NT;
  C pre[EPT];
  auto fetch = [&](int v0) {
    const int nv = min(V, vend - v0);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = t + NT * q;
      const int ww = e % W, j = (e / W) % NZ, v = e / (W * NZ);
      pre[q] = (v < nv && j < nzp && kx0 + ww < Lx) ? ld_stream(base + ((size_t)(v0 + v) * nzp + j) * plane + ww)
                                                   : C{0, 0};
    }
  };
  if (vbeg < vend) fetch(vbeg);
  for (int v0 = vbeg; v0 < vend; v0 += V) {
    const int nv = min(V, vend - v0);
    __syncthreads();  // previous chunk's readers are done with xs
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = t + NT * q;
      if (e < V * NZ * W) xs[e] = pre[q];
    }
    __syncthreads();
    if (v0 + V < vend) fetch(v0 + V);  // next chunk in flight during the sums
    for (int v = 0; v < nv; ++v) {
      T ar[R], ai[R];
#pragma unroll
      for (int r = 0; r < R; ++r) ar[r] = ai[r] = 0;
      const C* xv = xs + (size_t)v * NZ * W + w;
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        const C xj = xv[j * W];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          ar[r] += m[r][j] * xj.x;
          ai[r] += m[r][j] * xj.y;
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = rg + r * RG;
        if (i < nzp && valid) st_stream(base + ((size_t)(v0 + v) * nzp + i) * plane + w, C{ar[r], ai[r]});
      }
    }
  }
}

// ------------------------------- Z step, piecewise-linear basis (C = 5) --
// The five components of one right-hand side couple through the blocks of
// eq. 8.  With the xy-transformed family kernels G_f(kx, ky, z_j - z_i)
// (source minus observer plane; M1x and M1y are j times the stored real
// value, M1z is odd in the plane offset) and u = I2D + I3D, w = I2D - I3D,
// twelve z convolutions per pencil give all blocks:
//   a0..a2 = M0 * (Ix, Iy, Iz)   b0, b1 = M1x * (u, Ix)   c0, c1 = M1y * (w, Iy)
//   d0, d1 = M1z * (I3D, Iz)     e0, e1, e2 = M2x * u, M2y * w, M2z * I3D
//   y_x  = a0 + j b0            y_y = a1 - j c0          y_z = a2 - 2 d0
//   y_2D = j (c1 - b1) + e0 + e1
//   y_3D = -j (b1 + c1) + 2 d1 + e0 - e1 + 4 e2
// (block (x, 2D) = +M1x, (2D, x) = -M1x, ... as the basis definitions of
// eqs. 4-6 give them).  Block: W adjacent kx of one ky, RG row groups; the
// block's kernels G_f[slot][w] sit in LDS for all right-hand sides, one
// right-hand side's five components are staged in LDS at a time (the next
// one is in flight in registers) and updated in place.
template <typename T, int NZ, int RG>
__global__ void __launch_bounds__(256) k_zdirect5(Geo geo, int Lx, int Ly, int nzp, int nd, int nrhs, int rpb,
                                                  const uint8_t* __restrict__ qtab,
                                                  const T* __restrict__ g5,
                                                  typename CT<T>::t* __restrict__ B) {
  typedef typename CT<T>::t C;
  constexpr int W = 256 / RG;
  constexpr int R = (NZ + RG - 1) / RG;
  constexpr int NF = 7;
  extern __shared__ unsigned char smem_raw[];
  C* xs = reinterpret_cast<C*>(smem_raw);                  // [5][NZ][W]
  T* gs = reinterpret_cast<T*>(xs + (size_t)5 * NZ * W);   // [7][nd][W]
  const int t = threadIdx.x;
  const int ntile = (Lx + W - 1) / W;
  const int bid = first_item();  // XCD-aware order of the (tile, ky) blocks
  const int tile = bid % ntile, ky = bid / ntile;
  const int kx0 = tile * W;
  const int w = t % W, rg = t / W;
  const bool valid = kx0 + w < Lx;
  for (int e = t; e < NF * nd * W; e += 256) {
    const int ww = e % W, fq = e / W;
    gs[e] = kx0 + ww < Lx ? g5[((size_t)fq * Ly + ky) * Lx + kx0 + ww] : (T)0;
  }
  // offset-slot codes of this thread's rows, four per register
  uint32_t pk[R][(NZ + 3) / 4];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = rg + r * RG;
#pragma unroll
    for (int q = 0; q < (NZ + 3) / 4; ++q) {
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * q + b;
        const uint32_t c = (i < nzp && j < nzp) ? qtab[i * 32 + j] : 0u;
        v |= c << (8 * b);
      }
      pk[r][q] = v;
    }
  }
  const size_t plane = (size_t)geo.pb;
  C* base = B + (size_t)ky * geo.rp + kx0;
  const int rbeg = blockIdx.y * rpb;
  const int rend = min(nrhs, rbeg + rpb);
  constexpr int NE = 5 * NZ * W;
  constexpr int EPT = (NE + 255) / 256;
  C pre[EPT];
  auto fetch = [&](int rhs) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = t + 256 * q;
      const int ww = e % W, j = (e / W) % NZ, c = e / (W * NZ);
      pre[q] = (e < NE && j < nzp && kx0 + ww < Lx) ? ld_stream(base + ((size_t)(rhs * 5 + c) * nzp + j) * plane + ww)
                                                   : C{0, 0};
    }
  };
  if (rbeg < rend) fetch(rbeg);
  for (int rhs = rbeg; rhs < rend; ++rhs) {
    __syncthreads();  // previous right-hand side's readers are done with xs (and gs is loaded)
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = t + 256 * q;
      if (e < NE) xs[e] = pre[q];
    }
    __syncthreads();
    if (rhs + 1 < rend) fetch(rhs + 1);
    T acc[R][24];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < 24; ++k) acc[r][k] = 0;
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      if (j >= nzp) continue;
      const C ix = xs[(0 * NZ + j) * W + w];
      const C iy = xs[(1 * NZ + j) * W + w];
      const C iz = xs[(2 * NZ + j) * W + w];
      const C i2 = xs[(3 * NZ + j) * W + w];
      const C i3 = xs[(4 * NZ + j) * W + w];
      const C u = C{i2.x + i3.x, i2.y + i3.y};
      const C v = C{i2.x - i3.x, i2.y - i3.y};
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t code = (pk[r][j >> 2] >> (8 * (j & 3))) & 0xffu;
        const T* gq = gs + (code & 0x7fu) * W + w;
        const T g0 = gq[0 * nd * W], g1x = gq[1 * nd * W], g1y = gq[2 * nd * W];
        T g1z = gq[3 * nd * W];
        const T g2x = gq[4 * nd * W], g2y = gq[5 * nd * W], g2z = gq[6 * nd * W];
        if (code & 0x80u) g1z = -g1z;
        T* a = acc[r];
        a[0] += g0 * ix.x;  a[1] += g0 * ix.y;
        a[2] += g0 * iy.x;  a[3] += g0 * iy.y;
        a[4] += g0 * iz.x;  a[5] += g0 * iz.y;
        a[6] += g1x * u.x;  a[7] += g1x * u.y;
        a[8] += g1x * ix.x; a[9] += g1x * ix.y;
        a[10] += g1y * v.x; a[11] += g1y * v.y;
        a[12] += g1y * iy.x; a[13] += g1y * iy.y;
        a[14] += g1z * i3.x; a[15] += g1z * i3.y;
        a[16] += g1z * iz.x; a[17] += g1z * iz.y;
        a[18] += g2x * u.x; a[19] += g2x * u.y;
        a[20] += g2y * v.x; a[21] += g2y * v.y;
        a[22] += g2z * i3.x; a[23] += g2z * i3.y;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = rg + r * RG;
      if (i >= nzp || !valid) continue;
      const T* a = acc[r];
      // a0 = a[0,1], a1 = a[2,3], a2 = a[4,5], b0 = a[6,7], b1 = a[8,9],
      // c0 = a[10,11], c1 = a[12,13], d0 = a[14,15], d1 = a[16,17],
      // e0 = a[18,19], e1 = a[20,21], e2 = a[22,23]
      const C yx = C{a[0] - a[7], a[1] + a[6]};
      const C yy = C{a[2] + a[11], a[3] - a[10]};
      const C yz = C{a[4] - 2 * a[14], a[5] - 2 * a[15]};
      const C y2 = C{-(a[13] - a[9]) + a[18] + a[20], (a[12] - a[8]) + a[19] + a[21]};
      const C y3 = C{(a[9] + a[13]) + 2 * a[16] + a[18] - a[20] + 4 * a[22],
                     -(a[8] + a[12]) + 2 * a[17] + a[19] - a[21] + 4 * a[23]};
      C* o = base + ((size_t)(rhs * 5) * nzp + i) * plane + w;
      const size_t cs = (size_t)nzp * plane;
      st_stream(o, yx);
      st_stream(o + cs, yy);
      st_stream(o + 2 * cs, yz);
      st_stream(o + 3 * cs, y2);
      st_stream(o + 4 * cs, y3);
    }
  }
}

// --------------------------------------------------------------- Xi pass --
// FP32 with one pencil per wavefront: at least four 256-thread blocks per CU
// (at most 128 VGPRs), four waves per SIMD to cover the scatter's loads.
template <typename T, class P> struct XiMinBlocks {
  static constexpr int v = (sizeof(T) == 4 && wave_pencils<P>()) ? 4 : 1;
};
template <typename T, class P>
__global__ void __launch_bounds__(256, (XiMinBlocks<T, P>::v)) k_pass_xi(FftPlan pl, Geo geo, int WX, int Kx, int Ky, int nzp, int K, int nvec,
                                                  EpiParams ep, const XRowWord* __restrict__ xrow,
                                                  const typename CT<T>::t* __restrict__ A,
                                                  const typename CT<T>::t* __restrict__ x,
                                                  typename CT<T>::t* __restrict__ y,
                                                  const typename CT<T>::t* __restrict__ sconv,
                                                  const typename CT<T>::t* __restrict__ cdiag,
                                                  T inv_n,
                                                  const typename CT<T>::t* __restrict__ tw) {
  typedef typename CT<T>::t C;
  extern __shared__ unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int t = threadIdx.x;
  const int TPP = P::tpof(pl);
  const int j0 = t % TPP, w = t / TPP;
  const int NP = nzp * Ky;
  const int ngrp = (NP + WX - 1) / WX;
  const int Lx = P::Lof(pl);
  const int nw = (Kx + 63) >> 6;  // occupancy words per row
  auto where = [&](int item, int& vec, int& yy, int& zp, bool& valid) {
    vec = item / ngrp;
    const int pen = (item % ngrp) * WX + w;
    valid = pen < NP;
    const int pc = valid ? pen : 0;
    yy = pc % Ky;
    zp = pc / Ky;
  };
  auto mk_in = [&](int item) {
    int vec, yy, zp;
    bool valid;
    where(item, vec, yy, zp, valid);
    return ColIn<C>{A + ((size_t)vec * nzp + zp) * geo.pa + (size_t)yy * geo.rp, 1, Lx, valid};
  };
  auto mk_out = [&](int item) {
    int vec, yy, zp;
    bool valid;
    where(item, vec, yy, zp, valid);
    const int f = ep.fidx[vec / ep.C];
    const C scale = f >= 0 ? cscale(sconv[f], inv_n) : C{inv_n, 0};
    const C* cd = f >= 0 ? cdiag + (size_t)f * K : nullptr;
    const int rhs = vec / ep.C, comp = vec % ep.C;
    // 1 for the constant functions, 1/6 and 1/2 for the linear ones of eqs. 5-6
    const T mass = comp < 3 ? (T)1 : comp == 3 ? (T)(1.0 / 6.0) : (T)0.5;
    return XOut<C, T, uniform_rows<P>()>{y + (size_t)rhs * ep.ldy + (size_t)comp * K,
                                         x + (size_t)rhs * ep.ldx + (size_t)comp * K, cd,
                                         make_xrow<uniform_rows<P>()>(xrow, zp * Ky + yy, nw, Kx, valid), scale,
                                         mass};
  };
  Lds<C, false> acc{lds, WX, pencil_pitch(Lx), w};
  const C* twl = lds_twiddles(lds + (size_t)WX * pencil_pitch(Lx), tw, Lx);
  run_items<P, C, +1, false, wave_pencils<P>()>(pl, j0, ngrp * nvec, mk_in, mk_out, acc, twl);
}

// ------------------------------------------------------------- launcher ---
Geo make_geo(const svh_problem* p, size_t csize) {
  Geo g;
  g.rp = p->L[0] + (int)(128 / csize);
  g.pa = (long long)p->K[1] * g.rp + (long long)(256 / csize);
  g.pb = (long long)p->L[1] * g.rp + (long long)(256 / csize);
  return g;
}

// FP32 coupled five-component z step on the matrix cores.  Per pencil the z
// sum of each family is a real Toeplitz matrix T_f[i][j] = g_f(|z_i - z_j|)
// (with the z-odd sign for M1z) applied to every right-hand side: a dense
// (planes x planes) by (planes x columns) product, run as
// v_mfma_f32_16x16x4f32 with T_f as the A operand and the staged operands of
// 8 right-hand sides as the 16 B columns (column r: Re, r + 8: Im of
// right-hand side r).  The 17 blocks of eq. 8 take 12 products per pencil
// (the 2 of M1z and 4 of M2z folded into the staged kernel values): yx, yy,
// yz and the z-even part of y3 accumulate their products directly (with
// i u, -i w, -I3 formed per operand); R = M1x Ix, S = M1y Iy, P = M2x u,
// Q = M2y w are accumulated apart and combined per element afterwards:
//   y2 = i (S - R) + P + Q,   y3 += -i (R + S) + P - Q.
// A block is 8 pencils (one wavefront each, 64-byte runs along x) x all
// right-hand sides in batches of 8; operands and results pass through LDS.
// The A operands are gathered from the block's kernel values in LDS at each
// step (codes of the lane's (i, j) pairs held packed in registers), and the
// two 16-row tiles run one after the other, so a wavefront holds 32
// accumulators and four wavefronts fit on each SIMD.  Lane layout (wave64):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; result register v
// of lane l is D[4 (l / 16) + v][l % 16].
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix-core step and its result layout for each precision
template <typename T> struct Mfma16;
template <> struct Mfma16<float> {
  using v4 = f32x4_t;
  __device__ static v4 mac(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma16<double> {
  using v4 = f64x4_t;
  __device__ static v4 mac(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename T, int NZ, int W>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
k_zdirect5m(Geo geo, int Lx, int Ly, int nzp, int nd, int nrhs, const uint8_t* __restrict__ qtab,
            const T* __restrict__ g5, typename CT<T>::t* __restrict__ B) {
  using C = typename CT<T>::t;
  using M = Mfma16<T>;
  constexpr int NT = W * 64;          // one wavefront per pencil
  constexpr int RB = 8;               // right-hand sides per batch
  constexpr int RT = (NZ + 15) / 16;  // 16-row tiles of observer planes
  constexpr int KS = NZ / 4;          // 4-plane steps over source planes
  // values per (component, plane) row of xs: the pad puts consecutive planes
  // 64 (FP32) or 32 (FP64) bytes apart in the bank cycle
  constexpr int JS = W * RB * 2 + (sizeof(T) == 4 ? 16 : 8);
  constexpr int NF = 7;
  constexpr int EPT = 5 * NZ / 8;     // staged complex values per thread and batch
  constexpr int NCW = (RT * KS + 3) / 4;
  static_assert(NZ % 8 == 0 && NZ <= 24, "plane count");
  extern __shared__ __align__(16) unsigned char zsm_raw[];
  T* xs = reinterpret_cast<T*>(zsm_raw);    // [5][NZ][JS]: staged operands, then results
  T* gs = xs + (size_t)5 * NZ * JS;         // [W][7 nd + 1] kernel values of the block's pencils
  const int gp = NF * nd + 1;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int ntile = (Lx + W - 1) / W;
  const int bid = first_item();
  const int tile = bid % ntile, ky = bid / ntile;
  const int kx0 = tile * W;
  for (int e = t; e < NF * nd * W; e += NT) {
    const int ww = e % W, fs = e / W, f = fs / nd;
    const T sc = f == 3 ? T(2) : f == 6 ? T(4) : T(1);
    gs[ww * gp + fs] = kx0 + ww < Lx ? sc * g5[((size_t)fs * Ly + ky) * Lx + kx0 + ww] : T(0);
  }
  // codes of this lane's (i, j) = (16 rt + l % 16, 4 ks + l / 16), four per word
  uint32_t cw[NCW];
#pragma unroll
  for (int q = 0; q < NCW; ++q) cw[q] = 0u;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int i = 16 * rt + (lane & 15), j = 4 * ks + (lane >> 4), n = rt * KS + ks;
      const uint32_t code = (i < nzp && j < nzp) ? qtab[i * 32 + j] : 0u;
      cw[n >> 2] |= code << (8 * (n & 3));
    }
  const T* gw = gs + w * gp;
  const size_t plane = (size_t)geo.pb;
  C* base = B + (size_t)ky * geo.rp + kx0;
  const int col = lane & 15, part = col >> 3;
  const int bw = w * 16 + (col & 7) * 2;  // this lane's right-hand side and pencil within a plane row of xs
  const T sg = part ? T(1) : T(-1);
  // staging map: thread t moves pencil t % W of right-hand side (t / W) % 8 at
  // planes t / 8W + 8 h of every component (q = c NZ / 8 + h): runs of W
  // complex values along x
  const int sw = t % W, sr = (t / W) & 7, sj = t / (8 * W);
  const bool sx = kx0 + sw < Lx;
  T* const xst = xs + sj * JS + sw * 16 + sr * 2;
  const size_t cs = (size_t)nzp * plane;  // one component vector
  C v[EPT];
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    // the codes are redefined here so that the A-operand addresses derived from
    // them are formed at each step instead of being held across the batch loop
#pragma unroll
    for (int q = 0; q < NCW; ++q) asm volatile("" : "+v"(cw[q]));
    // every load is issued unconditionally from a valid address (right-hand
    // side and plane clamped; positions x >= Lx lie in the row padding) and
    // zeros are selected when the values are staged, so that the loads of a
    // batch are in flight together
    {
      const C* src = base + (size_t)min(r0 + sr, nrhs - 1) * 5 * cs + sw;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int c = q / (NZ / 8), h = q % (NZ / 8);
        v[q] = src[c * cs + (size_t)min(sj + 8 * h, nzp - 1) * plane];
      }
    }
    __syncthreads();  // the previous batch's results have left xs (and gs is written)
    const bool sv = sx && r0 + sr < nrhs;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int c = q / (NZ / 8), h = q % (NZ / 8);
      *reinterpret_cast<C*>(xst + (c * NZ + 8 * h) * JS) = (sv && sj + 8 * h < nzp) ? v[q] : C{T(0), T(0)};
    }
    __syncthreads();
    T o0[4][5];  // results of the first row tile, kept until every wavefront has read its operands
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      typename M::v4 yx = {T(0), T(0), T(0), T(0)}, yy = yx, yz = yx, y3 = yx, pr = yx, ps = yx, pp = yx, pq = yx;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        // one step's LDS reads at a time: keeps the register count at the occupancy target
        __builtin_amdgcn_sched_barrier(0);
        const int n = rt * KS + ks;
        const uint32_t code = (cw[n >> 2] >> (8 * (n & 3))) & 0xffu;
        const T* ga = gw + (code & 0x7fu);
        const T a0 = ga[0], a1 = ga[nd], a2 = ga[2 * nd], a4 = ga[4 * nd], a5 = ga[5 * nd], a6 = ga[6 * nd];
        const T a3 = (code & 0x80u) ? -ga[3 * nd] : ga[3 * nd];
        const T* xj = xs + (4 * ks + (lane >> 4)) * JS + bw;
        const T ix = xj[0 * NZ * JS + part], iy = xj[1 * NZ * JS + part], iz = xj[2 * NZ * JS + part];
        const C p2 = *reinterpret_cast<const C*>(xj + 3 * NZ * JS);
        const C p3 = *reinterpret_cast<const C*>(xj + 4 * NZ * JS);
        const T i2 = part ? p2.y : p2.x, i2s = part ? p2.x : p2.y;
        const T i3 = part ? p3.y : p3.x, i3s = part ? p3.x : p3.y;
        const T u = i2 + i3, wv = i2 - i3;
        const T iu = sg * (i2s + i3s);    // i u
        const T miw = -sg * (i2s - i3s); // -i w
        yx = M::mac(a0, ix, yx);
        yy = M::mac(a0, iy, yy);
        yz = M::mac(a0, iz, yz);
        pr = M::mac(a1, ix, pr);
        ps = M::mac(a2, iy, ps);
        y3 = M::mac(a3, iz, y3);
        pp = M::mac(a4, u, pp);
        pq = M::mac(a5, wv, pq);
        yx = M::mac(a1, iu, yx);
        yy = M::mac(a2, miw, yy);
        yz = M::mac(a3, -i3, yz);
        y3 = M::mac(a6, i3, y3);
      }
      T res[4][5];
#pragma unroll
      for (int vr = 0; vr < 4; ++vr) {
        const T d = ps[vr] - pr[vr], sm = pr[vr] + ps[vr];
        const T ds = __shfl_xor(d, 8), ss = __shfl_xor(sm, 8);  // the other part of the same element
        res[vr][0] = yx[vr];
        res[vr][1] = yy[vr];
        res[vr][2] = yz[vr];
        res[vr][3] = sg * ds + pp[vr] + pq[vr];
        res[vr][4] = y3[vr] - sg * ss + pp[vr] - pq[vr];
      }
      if (rt == 0) {
#pragma unroll
        for (int vr = 0; vr < 4; ++vr)
#pragma unroll
          for (int c = 0; c < 5; ++c) o0[vr][c] = res[vr][c];
      }
      if (rt == RT - 1) {
        __syncthreads();  // every wavefront has read its operands
#pragma unroll
        for (int r2 = 0; r2 < RT; ++r2)
#pragma unroll
          for (int vr = 0; vr < 4; ++vr) {
            const int i = 16 * r2 + M::row(lane, vr);
            if (i < nzp) {
              T* o = xs + i * JS + bw + part;
#pragma unroll
              for (int c = 0; c < 5; ++c) o[c * NZ * JS] = r2 == rt ? res[vr][c] : o0[vr][c];
            }
          }
      }
    }
    __syncthreads();
    C* dst = base + (size_t)(r0 + sr) * 5 * cs + (size_t)sj * plane + sw;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int c = q / (NZ / 8), h = q % (NZ / 8);
      if (sv && sj + 8 * h < nzp)
        dst[c * cs + (size_t)(8 * h) * plane] = *reinterpret_cast<const C*>(xst + (c * NZ + 8 * h) * JS);
    }
  }
}

// Direct z sum (occupied planes) or padded z FFT: the direct sum whenever it
// applies (at most 32 occupied planes; with five components also at most 64
// distinct plane offsets) unless the FFT is asked for.
bool use_zdirect(const svh_problem* p) {
  const int nzp = (int)p->zlist.size();
  if (p->zstep == SVH_ZSTEP_FFT) return false;
  if (p->C == 5) return nzp <= kMaxDirectPlanes && p->d_qtab != nullptr;
  return nzp <= kMaxDirectPlanes;
}

static int pencils_per_block_x(int tp) {
  int w = 256 / tp;
  return w < 1 ? 1 : w;
}

// Columns per block of the strided passes: full 128-byte rows of x-adjacent
// elements when possible, within 1024 threads and 64 KiB of LDS.
static int cols_per_block(int tp, int L, size_t csize) {
  int W = csize == 16 ? 8 : 16;
  const int maxt = csize == 16 ? 512 : 1024;
  while (W > 1 && (W * tp > maxt || (size_t)W * L * csize > 65536)) W /= 2;
  return W;
}

template <typename T>
hipError_t launch_matvec_chunk(const svh_problem* p, int nvec, const EpiParams& ep, const void* xv,
                               void* yv, void* Av, void* Bv, const void* zhat, hipStream_t s,
                               hipEvent_t* ev) {
  typedef typename CT<T>::t C;
  const bool dbl = sizeof(T) == 8;
  const C* x = static_cast<const C*>(xv);
  C* y = static_cast<C*>(yv);
  C* A = static_cast<C*>(Av);
  C* B = static_cast<C*>(Bv);
  const C* tw[3];
  for (int a = 0; a < 3; ++a)
    tw[a] = dbl ? reinterpret_cast<const C*>(p->d_tw64[a]) : reinterpret_cast<const C*>(p->d_tw32[a]);
  const int Kx = p->K[0], Ky = p->K[1];
  const int Lx = p->L[0], Ly = p->L[1];
  const int nzp = (int)p->zlist.size();
  const int K = p->nvox;
  const Tune& tn = p->tune[dbl ? SVH_FP64 : SVH_FP32];
  const Geo geo = make_geo(p, sizeof(C));
  if (ev) hipEventRecord(ev[0], s);
  // X
  with_plan(Lx, [&](auto tag) {
    using P = decltype(tag);
    const FftPlan& pl = p->plan[0];
    const int tp = P::tpof(pl);
    const int WX = pencils_per_block_x(tp);
    const int NP = nzp * Ky;
    const int nitems = ((NP + WX - 1) / WX) * nvec;
    const size_t sh = (size_t)WX * pencil_pitch(Lx) * sizeof(C) + twiddle_bytes(Lx, sizeof(C));
    const int g = persistent_grid((const void*)k_pass_x<T, P>, WX * tp, sh, nitems, p->ncu, tn.grid_mult[0]);
    hipLaunchKernelGGL((k_pass_x<T, P>), dim3(g), dim3(WX * tp), sh, s, pl, geo, WX, Kx, Ky, nzp, K, nvec,
                       ep.C, ep.ldx, p->d_xrow, x, A, tw[0]);
  });
  if (ev) hipEventRecord(ev[1], s);
  // Y forward
  with_plan(Ly, [&](auto tag) {
    using P = decltype(tag);
    const FftPlan& pl = p->plan[1];
    const int tp = P::tpof(pl);
    const int W = std::max(1, cols_per_block(tp, Ly, sizeof(C)) >> tn.ycols_shift[0]);
    const int nitems = ((Lx + W - 1) / W) * nzp * nvec;
    const size_t sh = (size_t)W * Ly * sizeof(C) + twiddle_bytes(Ly, sizeof(C));
    const int g = persistent_grid((const void*)k_pass_y<T, -1, P>, W * tp, sh, nitems, p->ncu, tn.grid_mult[1]);
    hipLaunchKernelGGL((k_pass_y<T, -1, P>), dim3(g), dim3(W * tp), sh, s, pl, geo, W, Lx, Ky, nzp, nvec, A, B,
                       tw[1]);
  });
  if (ev) hipEventRecord(ev[2], s);
  // Z step: padded FFT along z with the spectrum product, or the direct sum
  const bool zdirect = use_zdirect(p);
  if (!zdirect) {
    const hipError_t ez = launch_zfft<T>(p, nvec, B, zhat, s);
    if (ez != hipSuccess) return ez;
  } else if (p->C == 5) {
    // coupled five-component direct sum with the kernel values read from LDS
    // (25-32 planes); double: 8 pencils x 32 row groups
    // (one row each), float: 16 pencils x 16 row groups
    const int nd = (int)p->dzset.size();
    const int nrhs = nvec / 5;
    const int NZ = nzp <= 8 ? 8 : nzp <= 16 ? 16 : nzp <= 24 ? 24 : 32;
    auto go = [&](auto nzt, auto rgt) -> hipError_t {
      constexpr int NZc = decltype(nzt)::value, RGc = decltype(rgt)::value;
      constexpr int W = 256 / RGc;
      const int ntile = (Lx + W - 1) / W;
      const int nblk = ntile * Ly;
      int rpb = nrhs;
      while (rpb > 1 && (long long)nblk * ((nrhs + rpb - 1) / rpb) < 4096) rpb = (rpb + 1) / 2;
      dim3 grid(nblk, (nrhs + rpb - 1) / rpb);
      const size_t sh = (size_t)5 * NZc * W * sizeof(C) + (size_t)7 * nd * W * sizeof(T);
      if (sh > (size_t)p->max_lds) return hipErrorInvalidConfiguration;
      hipLaunchKernelGGL((k_zdirect5<T, NZc, RGc>), grid, dim3(256), sh, s, geo, Lx, Ly, nzp, nd, nrhs, rpb,
                         p->d_qtab, static_cast<const T*>(zhat), B);
      return hipSuccess;
    };
    using I8 = std::integral_constant<int, 8>;
    using I16 = std::integral_constant<int, 16>;
    using I24 = std::integral_constant<int, 24>;
    using I32 = std::integral_constant<int, 32>;
    using RGmax = std::integral_constant<int, sizeof(T) == 8 ? 32 : 16>;
    // up to 24 planes: matrix-core Toeplitz products (k_zdirect5m), 64-byte
    // runs along x (8 pencils per block in FP32, 4 in FP64); 32 planes would
    // not fit its registers and LDS
    auto gom = [&](auto nzt) -> hipError_t {
      constexpr int NZc = decltype(nzt)::value;
      constexpr int W5 = sizeof(T) == 4 ? 8 : 4;
      constexpr int JS5 = W5 * 16 + (sizeof(T) == 4 ? 16 : 8);
      const int nblk = ((Lx + W5 - 1) / W5) * Ly;
      const size_t sh = ((size_t)5 * NZc * JS5 + (size_t)W5 * (7 * nd + 1)) * sizeof(T);
      if (sh > (size_t)p->max_lds) return hipErrorInvalidConfiguration;
      hipLaunchKernelGGL((k_zdirect5m<T, NZc, W5>), dim3(nblk), dim3(W5 * 64), sh, s, geo, Lx, Ly, nzp, nd, nrhs,
                         p->d_qtab, static_cast<const T*>(zhat), B);
      return hipSuccess;
    };
    hipError_t ez;
    if (NZ <= 24) {
      switch (NZ) {
        case 8: ez = gom(I8{}); break;
        case 16: ez = gom(I16{}); break;
        default: ez = gom(I24{}); break;
      }
    } else {
      switch (NZ) {
        case 8: ez = go(I8{}, I8{}); break;
        case 16: ez = go(I16{}, I16{}); break;
        case 24: ez = go(I24{}, RGmax{}); break;
        default: ez = go(I32{}, RGmax{}); break;
      }
    }
    if (ez != hipSuccess) return ez;
  } else if (zdirect) {
    // 512 threads: double 32 pencils x 16 row groups, float 64 pencils x 8
    // row groups (512-byte runs of each plane row)
    constexpr int NT = 512;
    constexpr int RG = sizeof(T) == 8 ? 16 : 8;
    constexpr int W = NT / RG;
    constexpr int V = 4;
    const int ntile = (Lx + W - 1) / W;
    const int nblk = ntile * Ly;
    int vpb = nvec;
    while (vpb > V && (long long)nblk * ((nvec + vpb - 1) / vpb) < 4096) vpb = (vpb + 1) / 2;
    dim3 grid(nblk, (nvec + vpb - 1) / vpb);
    const int NZ = nzp <= 8 ? 8 : nzp <= 16 ? 16 : nzp <= 24 ? 24 : 32;
    const size_t sh = (size_t)V * NZ * W * sizeof(C) + (size_t)NZ * sizeof(int) + (size_t)NZ * NZ;
    if (sh > (size_t)p->max_lds) return hipErrorInvalidConfiguration;
    const T* gk = static_cast<const T*>(zhat);
    switch (NZ) {
      case 8: hipLaunchKernelGGL((k_zdirect<T, 8, RG, V, NT>), grid, dim3(NT), sh, s, geo, Lx, Ly, nzp, nvec, vpb,
                                 p->d_zlist, ep.zslot ? p->d_qtab : nullptr, gk, B); break;
      case 16: hipLaunchKernelGGL((k_zdirect<T, 16, RG, V, NT>), grid, dim3(NT), sh, s, geo, Lx, Ly, nzp, nvec, vpb,
                                  p->d_zlist, ep.zslot ? p->d_qtab : nullptr, gk, B); break;
      case 24: hipLaunchKernelGGL((k_zdirect<T, 24, RG, V, NT>), grid, dim3(NT), sh, s, geo, Lx, Ly, nzp, nvec, vpb,
                                  p->d_zlist, ep.zslot ? p->d_qtab : nullptr, gk, B); break;
      default: hipLaunchKernelGGL((k_zdirect<T, 32, RG, V, NT>), grid, dim3(NT), sh, s, geo, Lx, Ly, nzp, nvec, vpb,
                                  p->d_zlist, ep.zslot ? p->d_qtab : nullptr, gk, B); break;
    }
  }
  if (ev) hipEventRecord(ev[3], s);
  // Y inverse
  with_plan(Ly, [&](auto tag) {
    using P = decltype(tag);
    const FftPlan& pl = p->plan[1];
    const int tp = P::tpof(pl);
    const int W = std::max(1, cols_per_block(tp, Ly, sizeof(C)) >> tn.ycols_shift[1]);
    const int nitems = ((Lx + W - 1) / W) * nzp * nvec;
    const size_t sh = (size_t)W * Ly * sizeof(C) + twiddle_bytes(Ly, sizeof(C));
    const int g = persistent_grid((const void*)k_pass_y<T, +1, P>, W * tp, sh, nitems, p->ncu, tn.grid_mult[2]);
    hipLaunchKernelGGL((k_pass_y<T, +1, P>), dim3(g), dim3(W * tp), sh, s, pl, geo, W, Lx, Ky, nzp, nvec, B, A,
                       tw[1]);
  });
  if (ev) hipEventRecord(ev[4], s);
  // X inverse + epilogue
  with_plan(Lx, [&](auto tag) {
    using P = decltype(tag);
    const FftPlan& pl = p->plan[0];
    const int tp = P::tpof(pl);
    const int WX = pencils_per_block_x(tp);
    const int NP = nzp * Ky;
    const int nitems = ((NP + WX - 1) / WX) * nvec;
    const size_t sh = (size_t)WX * pencil_pitch(Lx) * sizeof(C) + twiddle_bytes(Lx, sizeof(C));
    const int g = persistent_grid((const void*)k_pass_xi<T, P>, WX * tp, sh, nitems, p->ncu, tn.grid_mult[3]);
    // the z steps leave no factor (the direct sum uses the z-space kernel,
    // the z FFT divides by Lz in its product): only the x and y transforms'
    const T inv_n = (T)(1.0 / ((double)p->L[0] * p->L[1]));
    const C* sc = dbl ? reinterpret_cast<const C*>(p->d_sconv64) : reinterpret_cast<const C*>(p->d_sconv32);
    const C* cd = dbl ? reinterpret_cast<const C*>(p->d_cdiag64) : reinterpret_cast<const C*>(p->d_cdiag32);
    hipLaunchKernelGGL((k_pass_xi<T, P>), dim3(g), dim3(WX * tp), sh, s, pl, geo, WX, Kx, Ky, nzp, K, nvec, ep,
                       p->d_xrow, A, x, y, sc, cd, inv_n, tw[0]);
  });
  if (ev) hipEventRecord(ev[5], s);
  return hipGetLastError();
}

template hipError_t launch_matvec_chunk<double>(const svh_problem*, int, const EpiParams&, const void*,
                                                void*, void*, void*, const void*, hipStream_t, hipEvent_t*);
template hipError_t launch_matvec_chunk<float>(const svh_problem*, int, const EpiParams&, const void*,
                                               void*, void*, void*, const void*, hipStream_t, hipEvent_t*);

}  // namespace svh
