// Batched 1D FFTs of lines held in LDS, for one workgroup.
//
// Layout: element i of line l sits at buf[l * ls + i * es].  The thread
// mapping puts the line index fastest, so with interleaved lines (es = number
// of lines, ls = 1) every wave touches consecutive LDS addresses.
//
// Algorithm: mixed-radix Stockham autosort, decimation in time, ping-pong
// between two LDS buffers.  For a stage with radix R and ns = product of the
// earlier radices, butterfly j reads x[j + m n/R] (m < R), multiplies by
// w^{m k} with k = j mod ns and w = exp(-2 pi i / (ns R)), and writes X_m to
// ((j - k) R + k) + m ns; the output is in natural order.  Only the forward
// transform (exp(-2 pi i jk/n), unnormalized) is provided: callers obtain the
// inverse as conj(FFT(conj(x))) by conjugating in their own loads and stores.
//
// Codelets: radix 2, 4, 8, 16 (4 x 4) and 18 (6 x 3) in closed form; odd primes use the symmetric form
// of a prime-length DFT (a_q = x_q + x_{R-q}, b_q = x_q - x_{R-q}), which takes
// (R-1)^2 real multiply-adds per pair of outputs instead of R^2 complex ones,
// with cos and sin read at a wave-uniform index (LDS broadcast).  3, 5 and 7
// are unrolled in registers; larger odd primes run a stage that spreads each
// butterfly's output pairs over the threads and reads its inputs from LDS.
//
// Twiddle table (built on the host, copied to LDS): for every stage with
// ns > 1 the factors w^{m k}, stored [m-1][k] so that the lanes of a wave,
// which hold consecutive k, read consecutive addresses; for every odd-radix
// stage the R roots exp(-2 pi i q / R).
#pragma once
#include "fcns_common.hpp"

namespace fcns {

constexpr int FFT_MAX_STAGES = 12;

struct FFTPlan {
  int n;
  int nst;
  int r[FFT_MAX_STAGES];
  int toff[FFT_MAX_STAGES];  // stage twiddles [m-1][k] (ns > 1), else -1
  int coff[FFT_MAX_STAGES];  // roots of unity of odd radices, else -1
  int tsize;                 // complex entries of the whole table
};

// ---------------------------------------------------------------- codelets
template <typename T>
__device__ __forceinline__ void dft4_reg(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  const cpx<T> s02 = a0 + a2, d02 = a0 - a2, s13 = a1 + a3;
  const cpx<T> d13 = mul_mi(a1 - a3);
  a0 = s02 + s13;
  a2 = s02 - s13;
  a1 = d02 + d13;
  a3 = d02 - d13;
}

template <typename T, int R>
struct Codelet;

template <typename T>
struct Codelet<T, 2> {
  __device__ __forceinline__ static void run(cpx<T>* v, const cpx<T>*) {
    const cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T>
struct Codelet<T, 4> {
  __device__ __forceinline__ static void run(cpx<T>* v, const cpx<T>*) {
    dft4_reg<T>(v[0], v[1], v[2], v[3]);
  }
};

template <typename T>
struct Codelet<T, 8> {
  __device__ __forceinline__ static void run(cpx<T>* v, const cpx<T>*) {
    // n = n1 + 4 n2: even outputs from a = x_n1 + x_n1+4, odd outputs from
    // b = (x_n1 - x_n1+4) w8^n1, w8 = exp(-i pi/4)
    const T h = T(0.70710678118654752440084436210484903928483593768847);
    cpx<T> a0 = v[0] + v[4], a1 = v[1] + v[5], a2 = v[2] + v[6], a3 = v[3] + v[7];
    cpx<T> b0 = v[0] - v[4], b1 = v[1] - v[5], b2 = v[2] - v[6], b3 = v[3] - v[7];
    b1 = mk((b1.x + b1.y) * h, (b1.y - b1.x) * h);
    b2 = mul_mi(b2);
    b3 = mk((b3.y - b3.x) * h, -(b3.x + b3.y) * h);
    dft4_reg<T>(a0, a1, a2, a3);
    dft4_reg<T>(b0, b1, b2, b3);
    v[0] = a0;
    v[2] = a1;
    v[4] = a2;
    v[6] = a3;
    v[1] = b0;
    v[3] = b1;
    v[5] = b2;
    v[7] = b3;
  }
};

// Roots w_N^m = cos(2 pi m / N) - i sin(2 pi m / N) of the composite codelets.
struct Roots16 {
  static constexpr double c[16] = {1.0, 0.9238795325112867561281832, 0.7071067811865475244008444,
                                   0.38268343236508977172846, 0.0, -0.38268343236508977172846,
                                   -0.7071067811865475244008444, -0.9238795325112867561281832,
                                   -1.0, -0.9238795325112867561281832,
                                   -0.7071067811865475244008444, -0.38268343236508977172846,
                                   0.0, 0.38268343236508977172846, 0.7071067811865475244008444,
                                   0.9238795325112867561281832};
  static constexpr double s[16] = {0.0, 0.38268343236508977172846, 0.7071067811865475244008444,
                                   0.9238795325112867561281832, 1.0, 0.9238795325112867561281832,
                                   0.7071067811865475244008444, 0.38268343236508977172846, 0.0,
                                   -0.38268343236508977172846, -0.7071067811865475244008444,
                                   -0.9238795325112867561281832, -1.0,
                                   -0.9238795325112867561281832, -0.7071067811865475244008444,
                                   -0.38268343236508977172846};
};
struct Roots18 {
  static constexpr double c[18] = {1.0, 0.9396926207859083840541093, 0.7660444431189780352023927,
                                   0.5, 0.1736481776669303488517166, -0.1736481776669303488517166,
                                   -0.5, -0.7660444431189780352023927, -0.9396926207859083840541093,
                                   -1.0, -0.9396926207859083840541093, -0.7660444431189780352023927,
                                   -0.5, -0.1736481776669303488517166, 0.1736481776669303488517166,
                                   0.5, 0.7660444431189780352023927, 0.9396926207859083840541093};
  static constexpr double s[18] = {0.0, 0.3420201433256687330440996, 0.6427876096865393263226434,
                                   0.8660254037844386467637232, 0.984807753012208059366743,
                                   0.984807753012208059366743, 0.8660254037844386467637232,
                                   0.6427876096865393263226434, 0.3420201433256687330440996, 0.0,
                                   -0.3420201433256687330440996, -0.6427876096865393263226434,
                                   -0.8660254037844386467637232, -0.984807753012208059366743,
                                   -0.984807753012208059366743, -0.8660254037844386467637232,
                                   -0.6427876096865393263226434, -0.3420201433256687330440996};
};

// v (cos - i sin)
template <typename T>
__device__ __forceinline__ cpx<T> rot(const cpx<T>& v, double c, double s) {
  return mk(v.x * (T)c + v.y * (T)s, v.y * (T)c - v.x * (T)s);
}

// 3-point DFT with constant roots (w3 = -1/2 - i sqrt(3)/2).
template <typename T>
__device__ __forceinline__ void dft3_reg(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2) {
  const T h = T(0.8660254037844386467637231707529361834714);
  const cpx<T> sm = a1 + a2, df = a1 - a2;
  const cpx<T> c = a0 - sm * T(0.5);
  const cpx<T> r = mk(df.y * h, -df.x * h);  // -i sqrt(3)/2 (a1 - a2)
  a0 = a0 + sm;
  a1 = c + r;
  a2 = c - r;
}

// 6-point DFT in place: 3-point DFTs of the even and odd samples, then
// X_k = E_k + w6^k O_k, X_{k+3} = E_k - w6^k O_k.
template <typename T>
__device__ __forceinline__ void dft6_reg(cpx<T>* a) {
  const double h = 0.8660254037844386467637231707529361834714;
  cpx<T> e0 = a[0], e1 = a[2], e2 = a[4], o0 = a[1], o1 = a[3], o2 = a[5];
  dft3_reg<T>(e0, e1, e2);
  dft3_reg<T>(o0, o1, o2);
  const cpx<T> t1 = rot(o1, 0.5, h), t2 = rot(o2, -0.5, h);
  a[0] = e0 + o0;
  a[3] = e0 - o0;
  a[1] = e1 + t1;
  a[4] = e1 - t1;
  a[2] = e2 + t2;
  a[5] = e2 - t2;
}

// Composite codelets by one Cooley-Tukey split N = N1 N2 (n = N2 n1 + n2,
// k = k1 + N1 k2): N2 inner DFTs of length N1, twiddles w_N^(n2 k1), N1
// outer DFTs of length N2; all in registers with constant roots.
// 16 = 4 x 4
template <typename T>
struct Codelet<T, 16> {
  __device__ __forceinline__ static void run(cpx<T>* v, const cpx<T>*) {
    cpx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
      dft4_reg<T>(a[n2][0], a[n2][1], a[n2][2], a[n2][3]);
    }
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1)
        a[n2][k1] = rot(a[n2][k1], Roots16::c[n2 * k1], Roots16::s[n2 * k1]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<T> b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
      dft4_reg<T>(b0, b1, b2, b3);
      v[k1] = b0;
      v[k1 + 4] = b1;
      v[k1 + 8] = b2;
      v[k1 + 12] = b3;
    }
  }
};

// 18 = 6 x 3
template <typename T>
struct Codelet<T, 18> {
  __device__ __forceinline__ static void run(cpx<T>* v, const cpx<T>*) {
    cpx<T> a[3][6];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < 6; ++n1) a[n2][n1] = v[3 * n1 + n2];
      dft6_reg<T>(a[n2]);
    }
#pragma unroll
    for (int n2 = 1; n2 < 3; ++n2)
#pragma unroll
      for (int k1 = 1; k1 < 6; ++k1)
        a[n2][k1] = rot(a[n2][k1], Roots18::c[n2 * k1], Roots18::s[n2 * k1]);
#pragma unroll
    for (int k1 = 0; k1 < 6; ++k1) {
      cpx<T> b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1];
      dft3_reg<T>(b0, b1, b2);
      v[k1] = b0;
      v[k1 + 6] = b1;
      v[k1 + 12] = b2;
    }
  }
};

// Odd prime P in registers.  cw: the P roots exp(-2 pi i q / P).  The inputs
// are consumed into the sums a and differences b before any output is
// written back, so the transform runs in place.
template <typename T, int P>
struct CodeletOdd {
  __device__ __forceinline__ static void run(cpx<T>* v, const cpx<T>* cw) {
    constexpr int H = (P - 1) / 2;
    cpx<T> a[H], b[H];
    const cpx<T> x0 = v[0];
    cpx<T> s = x0;
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      a[q - 1] = v[q] + v[P - q];
      b[q - 1] = v[q] - v[P - q];
      s = s + a[q - 1];
    }
    v[0] = s;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      cpx<T> re = x0, im = zero<T>();
#pragma unroll
      for (int q = 1; q <= H; ++q) {
        const cpx<T> w = cw[(q * k) % P];  // cos - i sin
        re = re + a[q - 1] * w.x;
        im = im + b[q - 1] * (-w.y);
      }
      // X_k = re - i im, X_{P-k} = re + i im
      v[k] = re + mul_mi(im);
      v[P - k] = re + mul_i(im);
    }
  }
};
template <typename T> struct Codelet<T, 3> : CodeletOdd<T, 3> {};
template <typename T> struct Codelet<T, 5> : CodeletOdd<T, 5> {};
template <typename T> struct Codelet<T, 7> : CodeletOdd<T, 7> {};

// j mod ns for 0 <= j < 2^24 without an integer division: the float quotient
// is off by at most one, which the two corrections absorb.
__device__ __forceinline__ int fast_mod(int j, int ns, float rcp) {
  const int q = (int)((float)j * rcp);
  int r = j - q * ns;
  r += (r < 0) ? ns : 0;
  r -= (r >= ns) ? ns : 0;
  return r;
}

// Position of element i of line l: l * ls + es * i, or with PAD one spare
// slot after every 8 elements, l * ls + es * (i + i / 8).  The padding makes
// the stride-R stores of the first stage hit distinct LDS banks when lines
// are contiguous (es = 1) or interleaved by fewer than 8 (es < 8); a padded
// line of n points spans es * (n + n / 8) slots.
template <bool PAD>
__device__ __forceinline__ int lds_pos(int l, int i, int es, int ls) {
  return l * ls + es * (PAD ? i + (i >> 3) : i);
}

// ---------------------------------------------------------------- one stage
template <typename T, int R, bool PAD>
__device__ __forceinline__ void fft_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                          int L, int es, int ls, int n, int ns,
                                          const cpx<T>* __restrict__ tws,
                                          const cpx<T>* __restrict__ cw, int tid, int nt) {
  const int nr = n / R;
  const int nb = L * nr;
  const float rcp = 1.0f / (float)ns;
  for (int g = tid; g < nb; g += nt) {
    const int l = g % L, j = g / L;
    const int k = fast_mod(j, ns, rcp);
    cpx<T> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = src[lds_pos<PAD>(l, j + m * nr, es, ls)];
    if (ns > 1) {
#pragma unroll
      for (int m = 1; m < R; ++m) v[m] = v[m] * tws[(m - 1) * ns + k];
    }
    Codelet<T, R>::run(v, cw);
    const int o = (j - k) * R + k;
#pragma unroll
    for (int m = 0; m < R; ++m) dst[lds_pos<PAD>(l, o + m * ns, es, ls)] = v[m];
  }
}

// Any odd prime R > 7 at run time, spread over the workgroup: a line of n
// points has only n / R butterflies of this radix, too few to occupy the
// threads, and one whole R-point DFT per thread would not fit in registers.
// Phase 1 twiddles the inputs in place (one thread per butterfly input);
// phase 2 gives each work item PG consecutive output pairs (X_k, X_{R-k}) of
// one butterfly (the first group also X_0), so that each input is read from
// LDS once per PG pairs.  The butterfly index is fastest across lanes, so the
// roots cw[q k mod R] are read at wave-uniform addresses.  PG = 5 where the
// stage has enough butterflies to keep half the workgroup busy, else one
// pair per item (small lines, e.g. 58 = 2 x 29, would otherwise idle most
// threads).
template <typename T, bool PAD, int PG>
__device__ __forceinline__ void prime_outputs(const cpx<T>* __restrict__ src,
                                              cpx<T>* __restrict__ dst, int R, int L, int es,
                                              int ls, int nr, int ns, float rcp,
                                              const cpx<T>* __restrict__ cw, int tid, int nt) {
  const int nb = L * nr;
  const int H = (R - 1) / 2;
  const int ngrp = (H + PG - 1) / PG;
  for (int g = tid; g < nb * (ngrp + (PG == 1 ? 1 : 0)); g += nt) {
    const int b = g % nb, grp = g / nb;
    const int l = b % L, j = b / L;
    const int k = fast_mod(j, ns, rcp);
    auto S = [&](int m) -> const cpx<T>& { return src[lds_pos<PAD>(l, j + m * nr, es, ls)]; };
    const int o = (j - k) * R + k;
    auto D = [&](int m) -> cpx<T>& { return dst[lds_pos<PAD>(l, o + m * ns, es, ls)]; };
    // PG = 1: item 0 of a butterfly is X_0 alone, item kk the pair kk
    const int k0 = (PG == 1) ? grp : 1 + grp * PG;
    const bool dc = (PG == 1) ? grp == 0 : grp == 0;
    const cpx<T> x0 = S(0);
    cpx<T> sum = x0, re[PG], im[PG];
    int qk[PG];
#pragma unroll
    for (int i = 0; i < PG; ++i) {
      re[i] = x0;
      im[i] = zero<T>();
      qk[i] = 0;
    }
    for (int q = 1; q <= H; ++q) {
      const cpx<T> xa = S(q), xb = S(R - q);
      const cpx<T> ps = xa + xb, ms = xa - xb;
      sum = sum + ps;
      if (PG == 1 && k0 == 0) continue;
#pragma unroll
      for (int i = 0; i < PG; ++i) {
        qk[i] += k0 + i;
        if (qk[i] >= R) qk[i] -= R;
        const cpx<T> w = cw[qk[i]];
        re[i] = re[i] + ps * w.x;
        im[i] = im[i] + ms * (-w.y);
      }
    }
    if (dc) D(0) = sum;
#pragma unroll
    for (int i = 0; i < PG; ++i) {
      const int kk = k0 + i;
      if (kk >= 1 && kk <= H) {
        D(kk) = re[i] + mul_mi(im[i]);
        D(R - kk) = re[i] + mul_i(im[i]);
      }
    }
  }
}

constexpr int PRIME_PG = 5;

template <typename T, bool PAD>
__device__ __forceinline__ void fft_stage_prime(cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                                int R, int L, int es, int ls, int n, int ns,
                                                const cpx<T>* __restrict__ tws,
                                                const cpx<T>* __restrict__ cw, int tid, int nt) {
  const int nr = n / R;
  const int nb = L * nr;
  const float rcp = 1.0f / (float)ns;
  if (ns > 1) {
    for (int g = tid; g < nb * (R - 1); g += nt) {
      const int b = g % nb, m = 1 + g / nb;
      const int l = b % L, j = b / L;
      const int k = fast_mod(j, ns, rcp);
      cpx<T>& x = src[lds_pos<PAD>(l, j + m * nr, es, ls)];
      x = x * tws[(m - 1) * ns + k];
    }
    __syncthreads();
  }
  const int H = (R - 1) / 2;
  if (2 * nb * ((H + PRIME_PG - 1) / PRIME_PG) >= nt)
    prime_outputs<T, PAD, PRIME_PG>(src, dst, R, L, es, ls, nr, ns, rcp, cw, tid, nt);
  else
    prime_outputs<T, PAD, 1>(src, dst, R, L, es, ls, nr, ns, rcp, cw, tid, nt);
}

// ---------------------------------------------------------------- driver
// Forward FFT of L lines of pl.n points.  The input is in buf0; buf1 is
// scratch of the same size; tw is the plan's twiddle table (in LDS).
// Returns the buffer holding the result.  All threads of the workgroup must
// call it, after a barrier that makes the input visible; it synchronises
// before returning.  BIG: also dispatch the run-time stage for odd primes
// above 7.  PAD: padded line layout (lds_pos).
template <typename T, int L, bool BIG, bool PAD = false>
__device__ __forceinline__ cpx<T>* fft_fwd(cpx<T>* buf0, cpx<T>* buf1, int es, int ls,
                                           const FFTPlan& pl, const cpx<T>* __restrict__ tw,
                                           int tid, int nt) {
  int ns = 1;
  const int n = pl.n;
  cpx<T>* src = buf0;
  cpx<T>* dst = buf1;
  for (int s = 0; s < pl.nst; ++s) {
    const int r = pl.r[s];
    const cpx<T>* tws = tw + (pl.toff[s] < 0 ? 0 : pl.toff[s]);
    const cpx<T>* cw = tw + (pl.coff[s] < 0 ? 0 : pl.coff[s]);
    switch (r) {
      case 2: fft_stage<T, 2, PAD>(src, dst, L, es, ls, n, ns, tws, cw, tid, nt); break;
      case 3: fft_stage<T, 3, PAD>(src, dst, L, es, ls, n, ns, tws, cw, tid, nt); break;
      case 4: fft_stage<T, 4, PAD>(src, dst, L, es, ls, n, ns, tws, cw, tid, nt); break;
      case 5: fft_stage<T, 5, PAD>(src, dst, L, es, ls, n, ns, tws, cw, tid, nt); break;
      case 7: fft_stage<T, 7, PAD>(src, dst, L, es, ls, n, ns, tws, cw, tid, nt); break;
      case 8: fft_stage<T, 8, PAD>(src, dst, L, es, ls, n, ns, tws, cw, tid, nt); break;
      default:
        if constexpr (BIG) fft_stage_prime<T, PAD>(src, dst, r, L, es, ls, n, ns, tws, cw, tid, nt);
        break;
    }
    __syncthreads();
    cpx<T>* t = src;
    src = dst;
    dst = t;
    ns *= r;
  }
  return src;
}

// ---------------------------------------------------------------- compile-time plans
// A transform length known at compile time: the radices (in the order the
// host plan builder uses, so the twiddle table layout is the same), and with
// them every stride, loop bound and modulus of a stage, which turns the index
// arithmetic of the run-time engine into shifts and constants.  DynPlan<BIG>
// selects the run-time engine instead.
template <int... Rs>
struct SPlan {
  static constexpr bool dynamic = false;
  static constexpr int n = (Rs * ... * 1);
  static constexpr int nst = sizeof...(Rs);
  static constexpr bool big = false;
};

template <bool BIG>
struct DynPlan {
  static constexpr bool dynamic = true;
  static constexpr int n = 0;
  static constexpr bool big = BIG;
};

template <typename T, int R, int NS, int N, int L, int NT, bool PAD>
__device__ __forceinline__ void sfft_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                           int es, int ls, const cpx<T>* __restrict__ tws,
                                           const cpx<T>* __restrict__ cw, int tid) {
  constexpr int NR = N / R;
  constexpr int NB = L * NR;
  constexpr int IT = (NB + NT - 1) / NT;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int g = tid + it * NT;
    if (NB % NT == 0 || g < NB) {
      const int l = g % L, j = g / L;
      const int k = j % NS;
      cpx<T> v[R];
#pragma unroll
      for (int m = 0; m < R; ++m) v[m] = src[lds_pos<PAD>(l, j + m * NR, es, ls)];
      if constexpr (NS > 1) {
#pragma unroll
        for (int m = 1; m < R; ++m) v[m] = v[m] * tws[(m - 1) * NS + k];
      }
      Codelet<T, R>::run(v, cw);
      const int o = (j - k) * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) dst[lds_pos<PAD>(l, o + m * NS, es, ls)] = v[m];
    }
  }
}

template <typename T, int L, int NT, bool PAD, int N, int S, int NS, int R, int... Rest>
__device__ __forceinline__ cpx<T>* sfft_from(cpx<T>* src, cpx<T>* dst, int es, int ls,
                                             const FFTPlan& pl, const cpx<T>* __restrict__ tw,
                                             int tid) {
  const cpx<T>* tws = tw + (NS > 1 ? pl.toff[S] : 0);
  const cpx<T>* cw = tw + ((R & 1) ? pl.coff[S] : 0);
  if constexpr (R % 2 == 1 && R > 8)  // odd primes: the cooperative stage, constant sizes
    fft_stage_prime<T, PAD>(src, dst, R, L, es, ls, N, NS, tws, cw, tid, NT);
  else
    sfft_stage<T, R, NS, N, L, NT, PAD>(src, dst, es, ls, tws, cw, tid);
  __syncthreads();
  if constexpr (sizeof...(Rest) == 0)
    return dst;
  else
    return sfft_from<T, L, NT, PAD, N, S + 1, NS * R, Rest...>(dst, src, es, ls, pl, tw, tid);
}

template <typename T, int L, int NT, bool PAD, int... Rs>
__device__ __forceinline__ cpx<T>* sfft(SPlan<Rs...>, cpx<T>* buf0, cpx<T>* buf1, int es, int ls,
                                        const FFTPlan& pl, const cpx<T>* __restrict__ tw, int tid) {
  return sfft_from<T, L, NT, PAD, SPlan<Rs...>::n, 0, 1, Rs...>(buf0, buf1, es, ls, pl, tw, tid);
}

// Forward FFT with plan FP (SPlan<...> or DynPlan<BIG>), NT threads; same
// contract as fft_fwd.
template <typename T, int L, int NT, bool PAD, class FP>
__device__ __forceinline__ cpx<T>* fft_run(cpx<T>* buf0, cpx<T>* buf1, int es, int ls,
                                           const FFTPlan& pl, const cpx<T>* __restrict__ tw,
                                           int tid) {
  if constexpr (FP::dynamic)
    return fft_fwd<T, L, FP::big, PAD>(buf0, buf1, es, ls, pl, tw, tid, NT);
  else
    return sfft<T, L, NT, PAD>(FP{}, buf0, buf1, es, ls, pl, tw, tid);
}

}  // namespace fcns
