// Periodic-direction kernels: FFTs along y (c2c) and x (r2c / c2r), and the
// fused x-pass that evaluates the advective products in physical space.
//
// Layouts (x fastest): physical real fields [planes][ny][nx]; (kx, y) and
// (kx, ky) complex fields [planes][ny][nkxp] holding nkx = nx/2 + 1 modes per
// row, the row stride nkxp padded to a multiple of 4 (64 B).  Inverse
// transforms use IFFT(y) = conj(FFT(conj(y))) / n with the conjugations folded
// into loads and stores.
#include "kernels.hpp"

#include <type_traits>

namespace fcns {

// ---------------------------------------------------------------- y pass
// Lines q = plane * nkxp + kx; a tile is YL consecutive lines, staged in LDS
// interleaved (element ky of line l at l + YL ky, y_span slots per buffer).  Each thread keeps one line of the tile (l = tid % YL,
// YNT being a multiple of YL) and the rows ky = tid / YL + r * YNT / YL.
// Workgroups loop over tiles and load the next tile into registers before
// transforming the current one, so the loads overlap the FFT.  mode 1
// (inverse only): a second pass transforms i k~y times the input into dst2.
// Lines are interleaved without padding: two workgroups of 512-point lines
// (2 x 4 lines x 512 points x 2 buffers) then fit the 160 KB of LDS per CU,
// which matters more than the 2-way bank conflicts of the first stage.
__host__ __device__ inline int y_span(int ny, int lines) { return lines * ny; }

size_t y_lds_bytes(int ny, int tsize, size_t elem, int lines) {
  return ((size_t)tsize + 2 * (size_t)y_span(ny, lines)) * elem;
}

bool y_wide_tiles(const YArgs& a) { return a.ny == 512 && plan_is(a.pl, {8, 8, 8}); }

// PF: load the next tile into registers while the current one is transformed
// (more registers, fewer waves per SIMD) or load each tile when it is needed.
// LT lines per tile, 64 LT threads (64 rows stepped per thread either way).
template <typename T, class FP, int OWN, bool PF, int LT>
__global__ __launch_bounds__(64 * LT) void k_y(YArgs a, const cpx<T>* src, cpx<T>* dst,
                                               cpx<T>* dst2, long long sfs, long long dfs,
                                               long long nlines, int inv, int mode) {
  constexpr int YL = LT, YNT = 64 * LT;
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int ny = FP::dynamic ? a.ny : FP::n;
  const int nkx = a.nkx, nkxp = a.nkxp;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + a.pl.tsize;
  cpx<T>* X1 = X0 + y_span(ny, YL);
  src += blockIdx.y * sfs;
  dst += blockIdx.y * dfs;
  if (mode == 1) dst2 += blockIdx.y * dfs;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < a.pl.tsize; i += YNT) tw[i] = gtw[i];
  const int l = tid % YL, ky0 = tid / YL;
  constexpr int KYS = YNT / YL;
  // the 512-point compiled plan keeps its first and last stages in registers
  constexpr bool RE = std::is_same<FP, SPlan<8, 8, 8>>::value && OWN == 8 && KYS == 64;
  const long long ntiles = (nlines + YL - 1) / YL;
  const T sc = inv ? T(1) / (T)ny : T(1);
  const int npass = (mode == 1) ? 2 : 1;
  cpx<T> cur[OWN], nxt[PF ? OWN : 1];
  // XCD-aware tile order: workgroups are dispatched to the 8 XCDs in turn
  // (workgroup b on XCD b % 8), and a tile is 4 kx columns, half of a
  // 128-byte line, so neighbouring tiles share lines.  Each round of G tiles
  // is cut into chunks of 64; in a chunk, XCD x takes the run of 8 tiles
  // 8x .. 8x + 7, one per workgroup of that XCD, so that neighbours meet
  // their shared lines in one L2 and a partial last round still spreads
  // over all XCDs.
  const long long G = gridDim.x;
  long long t = blockIdx.x;
  if (G % 64 == 0) {
    const int j = blockIdx.x / 8, x = blockIdx.x % 8;
    t = (long long)(j / 8) * 64 + x * 8 + j % 8;
  }
  // element ky of line (plane, kx) at base + ky * stride: row-major
  // (stride nkxp) or blocked (stride 4: the 4 columns of a tile contiguous)
  const bool sblk = a.blk & 1, dblk = a.blk & 2;
  const int sstr = sblk ? 4 : nkxp, dstr = dblk ? 4 : nkxp;
  auto line_at = [&](long long tt, bool& ok, bool blocked) {
    const long long q = tt * YL + l;
    const long long pl = q / nkxp, kx = q - pl * nkxp;
    ok = q < nlines && kx < nkx;
    if (!ok) return 0LL;
    return pl * ny * nkxp + (blocked ? (kx >> 2) * ny * 4 + (kx & 3) : kx);
  };
  auto line_base = [&](long long tt, bool& ok) { return line_at(tt, ok, sblk); };
  if constexpr (PF) {
    bool ok;
    const long long base = line_base(t, ok);
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int ky = ky0 + r * KYS;
      cur[r] = (ok && ky < ny) ? src[base + (long long)ky * sstr] : zero<T>();
    }
  }
  for (; t < ntiles; t += gridDim.x) {
    bool ok;
    const long long base = line_base(t, ok);
    const long long dbase = line_at(t, ok, dblk);
    if constexpr (PF) {
      bool okn;
      const long long basen = line_base(t + gridDim.x, okn);
#pragma unroll
      for (int r = 0; r < OWN; ++r) {
        const int ky = ky0 + r * KYS;
        nxt[r] = (okn && ky < ny) ? src[basen + (long long)ky * sstr] : zero<T>();
      }
    } else {
#pragma unroll
      for (int r = 0; r < OWN; ++r) {
        const int ky = ky0 + r * KYS;
        cur[r] = (ok && ky < ny) ? src[base + (long long)ky * sstr] : zero<T>();
      }
    }
    for (int pass = 0; pass < npass; ++pass) {
      if constexpr (RE) {
        // 512 = 8 x 8 x 8 with one butterfly per thread in every stage: the
        // first stage's inputs are this thread's rows ky0 + 64 m (its DFT
        // over m needs no twiddles), and so are the last stage's outputs.
        // Only the middle stage goes through LDS: two barriers per
        // transform.  Reuse of X0 / X1 by the next transform is ordered by
        // these barriers (a thread writes X0 only after the barrier that
        // ends every read of it, and X1 only after the next one).
        cpx<T> v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          cpx<T> x = cur[m];
          if (pass == 1) x = mul_i(x) * (T)k_odd(ky0 + 64 * m, 512, a.kys);
          v[m] = inv ? conj(x) : x;
        }
        Codelet<T, 8>::run(v, nullptr);
#pragma unroll
        for (int m = 0; m < 8; ++m) X0[lds_pos<false>(l, 8 * ky0 + m, YL, 1)] = v[m];
        __syncthreads();
        sfft_stage<T, 8, 8, 512, YL, YNT, false>(X0, X1, YL, 1, tw + a.pl.toff[1], nullptr, tid);
        __syncthreads();
        const cpx<T>* tws = tw + a.pl.toff[2];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = X1[lds_pos<false>(l, ky0 + 64 * m, YL, 1)];
#pragma unroll
        for (int m = 1; m < 8; ++m) v[m] = v[m] * tws[(m - 1) * 64 + ky0];
        Codelet<T, 8>::run(v, nullptr);
        cpx<T>* out = pass ? dst2 : dst;
        if (ok) {
#pragma unroll
          for (int m = 0; m < 8; ++m)
            out[dbase + (long long)(ky0 + 64 * m) * dstr] = (inv ? conj(v[m]) : v[m]) * sc;
        }
        continue;
      }
#pragma unroll
      for (int r = 0; r < OWN; ++r) {
        const int ky = ky0 + r * KYS;
        if (ky < ny) {
          cpx<T> v = cur[r];
          if (pass == 1) v = mul_i(v) * (T)k_odd(ky, ny, a.kys);
          X0[lds_pos<false>(l, ky, YL, 1)] = inv ? conj(v) : v;
        }
      }
      __syncthreads();
      const cpx<T>* R = fft_run<T, YL, YNT, false, FP>(X0, X1, YL, 1, a.pl, tw, tid);
      cpx<T>* out = pass ? dst2 : dst;
      if (ok) {
#pragma unroll
        for (int r = 0; r < OWN; ++r) {
          const int ky = ky0 + r * KYS;
          if (ky < ny) {
            const cpx<T> v = R[lds_pos<false>(l, ky, YL, 1)];
            out[dbase + (long long)ky * dstr] = (inv ? conj(v) : v) * sc;
          }
        }
      }
      __syncthreads();
    }
    if constexpr (PF) {
#pragma unroll
      for (int r = 0; r < OWN; ++r) cur[r] = nxt[r];
    }
  }
}

// ---------------------------------------------------------------- x helpers
// Rows r0..r0+XR-1; two real rows (2a, 2a+1) share complex line a:
// z[n] = x_2a[n] + i x_2a+1[n], staged in LDS line-contiguous with the padded
// layout of the FFT engine, element n of line a at xp(a, n) (line stride
// x_ls(nx) = 4 mod 8 slots, so the lines interleaved by the thread mapping
// fall on different banks).
constexpr int XL = XR / 2;

__host__ __device__ inline int x_ls(int nx) { return ((nx + nx / 8 + 7) / 8) * 8 + 4; }
__device__ __forceinline__ int xp(int a, int n, int ls) { return lds_pos<true>(a, n, 1, ls); }

// Pack the spectra A (row 2a), B (row 2a+1) of two real rows into the
// conjugate of the full spectrum of z = x_2a + i x_2a+1 (ready for the inverse
// via the conjugated forward transform).  The imaginary parts of the kx = 0
// and kx = nx/2 bins are dropped, as a c2r transform does.  dx: multiply by
// i k~x first.
template <typename T>
__device__ __forceinline__ void x_pack_c2r(cpx<T>* X, int ls, const cpx<double>* __restrict__ xy,
                                           long long r0, long long nrows, const XArgs& a,
                                           bool dx, int tid) {
  const int nx = a.nx, nkx = a.nkx, nkxp = a.nkxp;
#pragma unroll
  for (int al = 0; al < XL; ++al) {
    const long long ra = r0 + 2 * al, rb = ra + 1;
    for (int k = tid; k < nkx; k += XNT) {
      cpx<double> A = (ra < nrows) ? xy[ra * nkxp + k] : zero<double>();
      cpx<double> B = (rb < nrows) ? xy[rb * nkxp + k] : zero<double>();
      if (dx) {
        const double kx = (2 * k == nx) ? 0.0 : a.kxs * k;
        A = mul_i(A) * kx;
        B = mul_i(B) * kx;
      }
      if (k == 0 || 2 * k == nx) {
        A.y = 0.0;
        B.y = 0.0;
      }
      // Z[k] = A + i B, Z[nx - k] = conj(A) + i conj(B); store conjugates
      X[xp(al, k, ls)] = cvt<T>(conj(mk(A.x - B.y, A.y + B.x)));
      if (k > 0 && 2 * k < nx) X[xp(al, nx - k, ls)] = cvt<T>(conj(mk(A.x + B.y, B.x - A.y)));
    }
  }
}

// Unpack the forward transform of two packed real rows into their r2c spectra.
template <typename T>
__device__ __forceinline__ void x_unpack_r2c(const cpx<T>* X, int ls, cpx<double>* __restrict__ xy,
                                             long long r0, long long nrows, const XArgs& a,
                                             int tid) {
  const int nx = a.nx, nkx = a.nkx, nkxp = a.nkxp;
#pragma unroll
  for (int al = 0; al < XL; ++al) {
    const long long ra = r0 + 2 * al, rb = ra + 1;
    for (int k = tid; k < nkx; k += XNT) {
      const cpx<double> Z = cvt<double>(X[xp(al, k, ls)]);
      const cpx<double> Zm = conj(cvt<double>(X[xp(al, ((k == 0) ? 0 : nx - k), ls)]));
      if (ra < nrows) xy[ra * nkxp + k] = (Z + Zm) * 0.5;
      if (rb < nrows) xy[rb * nkxp + k] = mul_mi(Z - Zm) * 0.5;
    }
  }
}

// ---------------------------------------------------------------- x r2c / c2r
template <typename T, bool BIG>
__global__ __launch_bounds__(XNT) void k_x_r2c(XArgs a, const double* __restrict__ phys,
                                               cpx<double>* __restrict__ xy, long long pfs,
                                               long long xfs, long long nrows) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int nx = a.nx, ls = x_ls(nx);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + a.pl.tsize;
  cpx<T>* X1 = X0 + XL * ls;
  phys += blockIdx.y * pfs;
  xy += blockIdx.y * xfs;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < a.pl.tsize; i += XNT) tw[i] = gtw[i];
  const long long r0 = (long long)blockIdx.x * XR;
  T* Xs = reinterpret_cast<T*>(X0);
#pragma unroll
  for (int rl = 0; rl < XR; ++rl) {
    const long long r = r0 + rl;
    for (int n = tid; n < nx; n += XNT)
      Xs[2 * xp(rl >> 1, n, ls) + (rl & 1)] = (r < nrows) ? (T)phys[r * nx + n] : T(0);
  }
  __syncthreads();
  const cpx<T>* R = fft_fwd<T, XL, BIG, true>(X0, X1, 1, ls, a.pl, tw, tid, XNT);
  x_unpack_r2c<T>(R, ls, xy, r0, nrows, a, tid);
}

template <typename T, bool BIG>
__global__ __launch_bounds__(XNT) void k_x_c2r(XArgs a, const cpx<double>* __restrict__ xy,
                                               double* __restrict__ phys, long long xfs,
                                               long long pfs, long long nrows) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int nx = a.nx, ls = x_ls(nx);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + a.pl.tsize;
  cpx<T>* X1 = X0 + XL * ls;
  phys += blockIdx.y * pfs;
  xy += blockIdx.y * xfs;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < a.pl.tsize; i += XNT) tw[i] = gtw[i];
  const long long r0 = (long long)blockIdx.x * XR;
  x_pack_c2r<T>(X0, ls, xy, r0, nrows, a, false, tid);
  __syncthreads();
  const cpx<T>* R = fft_fwd<T, XL, BIG, true>(X0, X1, 1, ls, a.pl, tw, tid, XNT);
  const double sc = 1.0 / nx;
#pragma unroll
  for (int al = 0; al < XL; ++al) {
    const long long ra = r0 + 2 * al, rb = ra + 1;
    for (int n = tid; n < nx; n += XNT) {
      // z = conj(R) / nx: row 2a = Re z, row 2a+1 = Im z
      const cpx<T> z = R[xp(al, n, ls)];
      if (ra < nrows) phys[ra * nx + n] = (double)z.x * sc;
      if (rb < nrows) phys[rb * nx + n] = -(double)z.y * sc;
    }
  }
}

// ---------------------------------------------------------------- x pass with products
// NL_f = -(u dq_f/dx + v dq_f/dy + w dq_f/dz) at the physical points of RR
// rows (Sec. 4.2: derivatives in Fourier space, products in real space, no
// padding), then its r2c transform.  Passes: 0-2 physical u, v, w; then per
// field f: dq/dx, dq/dy, dq/dz (inverse), and the forward transform of NL_f.
// A workgroup of NT threads owns spectral columns k = tid + c NT and physical
// columns n = tid + c NT (c < CC, CC NT >= nx) of its RR rows; each thread
// loads the next pass's spectral inputs while the current pass is transformed.
template <typename T, class FP, int RR, int NT, int CC>
__global__ __launch_bounds__(NT) void k_x_nl(XArgs a, const cpx<T>* __restrict__ xyb,
                                             cpx<T>* __restrict__ nl, long long fs,
                                             long long nrows, int nfields) {
  constexpr int LL = RR / 2;
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  // with a compile-time plan every row length below is a constant
  const int nx = FP::dynamic ? a.nx : FP::n;
  const int nkx = nx / 2 + 1, nkxp = (nkx + 3) / 4 * 4, ls = x_ls(nx);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + a.pl.tsize;
  cpx<T>* X1 = X0 + LL * ls;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < a.pl.tsize; i += NT) tw[i] = gtw[i];
  const long long r0 = (long long)blockIdx.x * RR;
  const T sc = T(1) / (T)nx;
  T U[3][CC][RR];
  T acc[CC][RR];
  cpx<T> in[CC][RR];
  // source slot of c2r pass p (-1: forward pass)
  auto slot = [&](int p) {
    if (p < 3) return 3 * p;
    const int f = (p - 3) >> 2, kk = (p - 3) & 3;
    return kk == 3 ? -1 : 3 * f + (kk == 0 ? 0 : kk);
  };
  auto load = [&](int p) {
    const int sl = slot(p);
    if (sl < 0) return;
    const cpx<T>* src = xyb + sl * fs;
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      const int k = tid + c * NT;
#pragma unroll
      for (int r = 0; r < RR; ++r)
        in[c][r] = (k < nkx && r0 + r < nrows) ? src[(r0 + r) * nkxp + k] : zero<T>();
    }
  };
  const int npass = 3 + 4 * nfields;
  load(0);
  for (int pass = 0; pass < npass; ++pass) {
    const int f = (pass - 3) >> 2, kk = (pass - 3) & 3;
    const bool fwd = pass >= 3 && kk == 3;
    if (!fwd) {
      const bool dx = pass >= 3 && kk == 0;
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int k = tid + c * NT;
        if (k < nkx) {
          const T kx = (2 * k == nx) ? T(0) : (T)(a.kxs * k);
#pragma unroll
          for (int al = 0; al < LL; ++al) {
            cpx<T> A = in[c][2 * al], B = in[c][2 * al + 1];
            if (dx) {
              A = mul_i(A) * kx;
              B = mul_i(B) * kx;
            }
            if (k == 0 || 2 * k == nx) {
              A.y = T(0);
              B.y = T(0);
            }
            // Z[k] = A + i B, Z[nx - k] = conj(A) + i conj(B); stored conjugated
            X0[xp(al, k, ls)] = conj(mk(A.x - B.y, A.y + B.x));
            if (k > 0 && 2 * k < nx) X0[xp(al, nx - k, ls)] = conj(mk(A.x + B.y, B.x - A.y));
          }
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int n = tid + c * NT;
        if (n < nx) {
#pragma unroll
          for (int al = 0; al < LL; ++al)
            X0[xp(al, n, ls)] = mk(acc[c][2 * al], acc[c][2 * al + 1]);
        }
      }
    }
    // next pass's spectral inputs, in flight during this pass's transform
    int pn = pass + 1;
    if (pn < npass && slot(pn) < 0) ++pn;
    if (pn < npass) load(pn);
    __syncthreads();
    const cpx<T>* R = fft_run<T, LL, NT, true, FP>(X0, X1, 1, ls, a.pl, tw, tid);
    if (!fwd) {
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int n = tid + c * NT;
        if (n >= nx) continue;
        T v[RR];
#pragma unroll
        for (int al = 0; al < LL; ++al) {
          const cpx<T> z = R[xp(al, n, ls)];
          v[2 * al] = z.x * sc;
          v[2 * al + 1] = -z.y * sc;
        }
        if (pass < 3) {
#pragma unroll
          for (int r = 0; r < RR; ++r) {
            if (pass == 0) U[0][c][r] = v[r];
            else if (pass == 1) U[1][c][r] = v[r];
            else U[2][c][r] = v[r];
          }
        } else {
#pragma unroll
          for (int r = 0; r < RR; ++r) {
            const T u = (kk == 0) ? U[0][c][r] : ((kk == 1) ? U[1][c][r] : U[2][c][r]);
            if (kk == 0) acc[c][r] = -u * v[r];
            else acc[c][r] -= u * v[r];
          }
        }
      }
    } else {
      // unpack the r2c spectra of the RR rows
#pragma unroll
      for (int al = 0; al < LL; ++al) {
        const long long ra = r0 + 2 * al, rb = ra + 1;
        cpx<T>* dst = nl + f * fs;
        for (int k = tid; k < nkx; k += NT) {
          const cpx<T> Z = R[xp(al, k, ls)];
          const cpx<T> Zm = conj(R[xp(al, ((k == 0) ? 0 : nx - k), ls)]);
          if (ra < nrows) dst[ra * nkxp + k] = (Z + Zm) * T(0.5);
          if (rb < nrows) dst[rb * nkxp + k] = mul_mi(Z - Zm) * T(0.5);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- x pass, wave-level rows
// Rows of N = 512, 256, 192, 128, 96, 64 or 32 points with 8 points per
// lane: a row occupies S = N / 8 lanes (one row per wavefront at 512, two at
// 256 and 192, four at 128, five at 96, eight at 64, sixteen at 32), and
// lane t of a row (t < S) holds index t + S m (m = 0..7) of every
// transform, in and out.
//
// N = 512 = 8 x 8 x 8: n = n0 + 8 n1 + 64 n2, k = k0 + 8 k1 + 64 k2 (t = n0 + 8 n1):
//   a radix-8 DFT over n2 in registers, twiddle w64^(n1 k0);
//   exchange so that lane n0 + 8 k0 holds n1 = 0..7, radix-8 over n1,
//   twiddle w512^(n0 (k0 + 8 k1));
//   exchange so that lane k0 + 8 k1 holds n0 = 0..7, radix-8 over n0,
// which leaves X[t + 64 k2] in lane t.
// N = 256 = 8 x 32: n = t + 32 m, k = a + 8 b:
//   a radix-8 DFT over m in registers, twiddle w256^(t a);
//   the eight 32-point DFTs over t = t0 + 4 t1 (b = j1 + 8 j0): exchange so
//   that lane t0 + 4 a holds t1 = 0..7, radix-8 over t1, twiddle w32^(t0 j1);
//   exchange so that lane L holds t0 = 0..3 of c = a + 8 j1 = L and L + 32,
//   two radix-4 DFTs over t0,
// which leaves X[c + 64 j0] = X[L + 32 (h + 2 j0)] (c = L + 32 h) in lane L.
// N = 128 = 8 x 16: n = t + 16 m, k = a + 8 b:
//   a radix-8 DFT over m in registers, twiddle w128^(t a);
//   the eight 16-point DFTs over t = h + 2 t1 (b = j + 8 c): exchange so that
//   lane 2 a + h holds t1 = 0..7, radix-8 over t1, twiddle w16^(h j);
//   exchange so that lane a + 8 j0 holds, for j = j0 + 2 j1 (j1 = 0..3),
//   both halves h of output j, and a radix-2 DFT over h,
// which leaves X[a + 8 j + 64 c] = X[L + 16 (j1 + 4 c)] in lane L.
// N = 64 = 8 x 8: a radix-8 DFT over m, twiddle w64^(t a), one exchange so
// that lane a holds t = 0..7, radix-8 over t: X[a + 8 b] in lane a.
// N = 32 = 8 x 4: a radix-8 DFT over m, twiddle w32^(t a), one exchange so
// that lane L holds t = 0..3 of a = 2L and 2L + 1, two radix-4 DFTs, and a
// last exchange into natural order.
// N = 192 = 8 x 24 and 96 = 8 x 12 (S = 24, 12 lanes; 2 and 5 rows per
// wavefront, the 64 mod S spare lanes repeat a row's last lanes and store
// nothing): a radix-8 DFT over m, twiddle wN^(t a); the S-point DFTs over
// t = h + 3 t1 (b = j + (S/3) c): exchange so that a lane holds, for its
// (a, h), t1 = 0..S/3-1 (at 96 two values of a per lane), radix-8 (192) or
// two radix-4 (96) DFTs over t1, twiddle wS^(h j); exchange, radix-3 DFTs
// over h (X[a + 8 j + (8 S/3) c], c = 0..2) spread over the lanes, and a
// last exchange into natural order.
// The exchanges go through a padded per-row LDS buffer (conflict-free
// 16-byte accesses) and need only wave-level ordering, no workgroup barrier.
// Two real transforms share one complex transform: z = a + i b (inverse from
// the spectra A, B; forward of two nonlinear terms).
constexpr int XW_WAVES = 4;        // waves per workgroup
constexpr int XW_BUF = 512 + 64;   // padded slots of one wave's exchange buffer(s)

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Padded slots, written with the per-lane part separate so that the
// per-register part is an instruction offset.  N = 512: element
// 64 n0 + 8 k0 + n1 of exchange 1 sits at 65 n0 + 8 k0 + n1, element
// 8 j + n0 of exchange 2 at 9 j + n0.  N = 256: element (a, t) of exchange 1
// at 36 a + t, element (c, t0) of exchange 2 at 4 c + c / 4 + t0.  Both: element
// i of the natural-order buffer at i + i / 8.
__device__ __forceinline__ int xw_nat(int i) { return i + (i >> 3); }

// Per-lane twiddles, stored [register][t] in LDS (read at t + offset).
// N = 512: tw[k0 - 1][t] = w64^(n1 k0) (k0 = 1..7) with t = n0 + 8 n1, and
// tw[7 + k1][t] = w512^(n0 (k0' + 8 k1)) with t = n0 + 8 k0'.
// N = 256: tw[a - 1][t] = w256^(t a) (a = 1..7), tw[6 + j1][t] = w32^(t0 j1)
// (j1 = 1..7) with t = t0 + 4 a.  N = 128: tw[a - 1][t] = w128^(t a),
// tw[6 + j][L] = w16^(h j) with h = L & 1.  N = 64: tw[a - 1][t] = w64^(t a).
// N = 192, 96: tw[a - 1][t] = wN^(t a), tw[6 + j][L] = w(N/8)^(h j) with
// h = L mod 3.  N = 32: tw[a - 1][t] = w32^(t a).
constexpr int XW_TW = 15 * 64;

template <typename T, int N>
__device__ __forceinline__ void xw_twiddles(cpx<T>* tw, int tid) {
  constexpr int S = N / 8, NTW = (N == 512 ? 15 : 14) * S;
  static_assert(NTW <= XW_TW, "twiddle table");
  for (int e = tid; e < NTW; e += 64 * XW_WAVES) {
    const int reg = e / S, t = e % S;
    int j;  // power of wN
    if (N == 512)
      j = reg < 7 ? 8 * (t >> 3) * (reg + 1) : (t & 7) * ((t >> 3) + 8 * (reg - 7));
    else if (N == 256)
      j = reg < 7 ? t * (reg + 1) : 8 * (t & 3) * (reg - 6);
    else if (N == 128)   // tw[6 + j][L] = w16^(h j), h = L & 1
      j = reg < 7 ? t * (reg + 1) : 8 * (t & 1) * (reg - 6);
    else if (N == 192 || N == 96)   // tw[6 + j][L] = w(N/8)^(h j), h = L mod 3
      j = reg < 7 ? t * (reg + 1) : 8 * (t % 3) * (reg - 6);
    else
      j = reg < 7 ? t * (reg + 1) : 0;
    double sn, cs;
    sincospi(2.0 * j / N, &sn, &cs);
    tw[e] = mk((T)cs, (T)(-sn));   // exp(-2 pi i j / N)
  }
}

template <typename T>
__device__ __forceinline__ void wave_fft512(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                            const cpx<T>* __restrict__ tw, int lane) {
  const int n0 = lane & 7, hi = lane >> 3;  // hi = n1 before, k0 after exchange 1
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int k0 = 1; k0 < 8; ++k0) r[k0] = r[k0] * tw[(k0 - 1) * 64 + lane];
  cpx<T>* w1 = buf + 65 * n0 + hi;
#pragma unroll
  for (int k0 = 0; k0 < 8; ++k0) w1[8 * k0] = r[k0];
  wave_sync();
  const cpx<T>* r1 = buf + 65 * n0 + 8 * hi;
#pragma unroll
  for (int n1 = 0; n1 < 8; ++n1) r[n1] = r1[n1];
  wave_sync();
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int k1 = 0; k1 < 8; ++k1) r[k1] = r[k1] * tw[(7 + k1) * 64 + lane];
  cpx<T>* w2 = buf + 9 * hi + n0;
#pragma unroll
  for (int k1 = 0; k1 < 8; ++k1) w2[72 * k1] = r[k1];
  wave_sync();
  const cpx<T>* r2 = buf + 9 * lane;
#pragma unroll
  for (int q = 0; q < 8; ++q) r[q] = r2[q];
  wave_sync();
  Codelet<T, 8>::run(r, nullptr);
}

template <typename T>
__device__ __forceinline__ void wave_fft256(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                            const cpx<T>* __restrict__ tw, int t) {
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int a = 1; a < 8; ++a) r[a] = r[a] * tw[(a - 1) * 32 + t];
  cpx<T>* w1 = buf + t;
#pragma unroll
  for (int a = 0; a < 8; ++a) w1[36 * a] = r[a];
  wave_sync();
  const int t0 = t & 3, a = t >> 2;  // the lane's (t0, a) after exchange 1
  const cpx<T>* r1 = buf + 36 * a + t0;
#pragma unroll
  for (int t1 = 0; t1 < 8; ++t1) r[t1] = r1[4 * t1];
  wave_sync();
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int j1 = 1; j1 < 8; ++j1) r[j1] = r[j1] * tw[(6 + j1) * 32 + t];
  // c = a + 8 j1: 4 c + c / 4 + t0 = (4 a + a / 4 + t0) + 34 j1
  cpx<T>* w2 = buf + 4 * a + (a >> 2) + t0;
#pragma unroll
  for (int j1 = 0; j1 < 8; ++j1) w2[34 * j1] = r[j1];
  wave_sync();
  // c = t + 32 h: 4 c + c / 4 = (4 t + t / 4) + 136 h
  const cpx<T>* r2 = buf + 4 * t + (t >> 2);
  cpx<T> q[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) q[i] = r2[136 * (i >> 2) + (i & 3)];
  wave_sync();
  dft4_reg<T>(q[0], q[1], q[2], q[3]);
  dft4_reg<T>(q[4], q[5], q[6], q[7]);
  // q[4 h + j0] = X[t + 32 (h + 2 j0)]
#pragma unroll
  for (int m = 0; m < 8; ++m) r[m] = q[4 * (m & 1) + (m >> 1)];
}

template <typename T>
__device__ __forceinline__ void wave_fft128(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                            const cpx<T>* __restrict__ tw, int t) {
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int a = 1; a < 8; ++a) r[a] = r[a] * tw[(a - 1) * 16 + t];
  // exchange 1: element (a, t) at 17 a + t
  cpx<T>* w1 = buf + t;
#pragma unroll
  for (int a = 0; a < 8; ++a) w1[17 * a] = r[a];
  wave_sync();
  const int a = t >> 1, h = t & 1;  // the lane's (a, h) after exchange 1
  const cpx<T>* r1 = buf + 17 * a + h;
#pragma unroll
  for (int t1 = 0; t1 < 8; ++t1) r[t1] = r1[2 * t1];
  wave_sync();
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int j = 1; j < 8; ++j) r[j] = r[j] * tw[(6 + j) * 16 + t];
  // exchange 2: output j of lane L = 2 a + h at 9 L + j
  cpx<T>* w2 = buf + 9 * t;
#pragma unroll
  for (int j = 0; j < 8; ++j) w2[j] = r[j];
  wave_sync();
  const int a2 = t & 7, j0 = t >> 3;
  const cpx<T>* r2 = buf + 18 * a2 + j0;
#pragma unroll
  for (int j1 = 0; j1 < 4; ++j1) {
    const cpx<T> p0 = r2[2 * j1], p1 = r2[9 + 2 * j1];
    r[j1] = p0 + p1;
    r[j1 + 4] = p0 - p1;
  }
  wave_sync();
}

template <typename T>
__device__ __forceinline__ void wave_fft64(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                           const cpx<T>* __restrict__ tw, int t) {
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int a = 1; a < 8; ++a) r[a] = r[a] * tw[(a - 1) * 8 + t];
  // element (a, t) at 9 a + t; lane a then reads t = 0..7
  cpx<T>* w1 = buf + t;
#pragma unroll
  for (int a = 0; a < 8; ++a) w1[9 * a] = r[a];
  wave_sync();
  const cpx<T>* r1 = buf + 9 * t;
#pragma unroll
  for (int t1 = 0; t1 < 8; ++t1) r[t1] = r1[t1];
  wave_sync();
  Codelet<T, 8>::run(r, nullptr);
}

// Outputs of the N = 192 and 96 transforms: P_h[a][j] (twiddled) sits at
// PS h + b, b = a + 8 j < Q = 8 S / 3; lane t takes the radix-3 DFTs over h
// of b = t, t + S, ... (< Q), X[b + Q c] for c = 0, 1, 2, writes them in
// natural order (slots xw_nat), and reads back its own X[t + S m].
template <typename T, int S, int PS>
__device__ __forceinline__ void xw_radix3_out(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                              int t) {
  constexpr int Q = 8 * S / 3;          // radix-3 DFTs per row (64 at 192, 32 at 96)
  constexpr int NB = (Q + S - 1) / S;   // per lane, the last one partial
  const T s3 = T(0.86602540378443864676);  // sqrt(3) / 2
  cpx<T> o[3 * NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + S * i;
    if (b < Q) {
      const cpx<T> p0 = buf[b], p1 = buf[PS + b], p2 = buf[2 * PS + b];
      const cpx<T> sm = p1 + p2, df = p1 - p2;
      const cpx<T> e = mul_i(df) * s3;
      const cpx<T> base = p0 - sm * T(0.5);
      o[3 * i] = p0 + sm;
      o[3 * i + 1] = base - e;   // w3 = -1/2 - i sqrt(3)/2
      o[3 * i + 2] = base + e;
    }
  }
  wave_sync();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + S * i;
    if (b < Q) {
#pragma unroll
      for (int c = 0; c < 3; ++c) buf[xw_nat(b + Q * c)] = o[3 * i + c];
    }
  }
  wave_sync();
#pragma unroll
  for (int m = 0; m < 8; ++m) r[m] = buf[xw_nat(t + S * m)];
}

template <typename T>
__device__ __forceinline__ void wave_fft192(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                            const cpx<T>* __restrict__ tw, int t) {
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int a = 1; a < 8; ++a) r[a] = r[a] * tw[(a - 1) * 24 + t];
  // exchange 1: element (a, t) at 25 a + t; lane 3 a + h reads t = h + 3 t1
  cpx<T>* w1 = buf + t;
#pragma unroll
  for (int a = 0; a < 8; ++a) w1[25 * a] = r[a];
  wave_sync();
  const int a = t / 3, h = t - 3 * a;
  const cpx<T>* r1 = buf + 25 * a + h;
#pragma unroll
  for (int t1 = 0; t1 < 8; ++t1) r[t1] = r1[3 * t1];
  wave_sync();
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int j = 1; j < 8; ++j) r[j] = r[j] * tw[(6 + j) * 24 + t];
  // exchange 2: P_h[a][j] at 65 h + a + 8 j
  cpx<T>* w2 = buf + 65 * h + a;
#pragma unroll
  for (int j = 0; j < 8; ++j) w2[8 * j] = r[j];
  wave_sync();
  xw_radix3_out<T, 24, 65>(r, buf, t);
  wave_sync();
}

template <typename T>
__device__ __forceinline__ void wave_fft96(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                           const cpx<T>* __restrict__ tw, int t) {
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int a = 1; a < 8; ++a) r[a] = r[a] * tw[(a - 1) * 12 + t];
  // exchange 1: element (a, t) at 13 a + t; lane 3 ap + h reads t = h + 3 t1
  // of a = 2 ap (registers 0..3) and 2 ap + 1 (registers 4..7)
  cpx<T>* w1 = buf + t;
#pragma unroll
  for (int a = 0; a < 8; ++a) w1[13 * a] = r[a];
  wave_sync();
  const int ap = t / 3, h = t - 3 * ap;
  const cpx<T>* r1 = buf + 26 * ap + h;
#pragma unroll
  for (int t1 = 0; t1 < 4; ++t1) {
    r[t1] = r1[3 * t1];
    r[4 + t1] = r1[13 + 3 * t1];
  }
  wave_sync();
  dft4_reg(r[0], r[1], r[2], r[3]);
  dft4_reg(r[4], r[5], r[6], r[7]);
#pragma unroll
  for (int j = 1; j < 4; ++j) {
    const cpx<T> f = tw[(6 + j) * 12 + t];
    r[j] = r[j] * f;
    r[4 + j] = r[4 + j] * f;
  }
  // exchange 2: P_h[a][j] at 33 h + a + 8 j
  cpx<T>* w2 = buf + 33 * h + 2 * ap;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    w2[8 * j] = r[j];
    w2[8 * j + 1] = r[4 + j];
  }
  wave_sync();
  xw_radix3_out<T, 12, 33>(r, buf, t);
  wave_sync();
}

template <typename T>
__device__ __forceinline__ void wave_fft32(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                           const cpx<T>* __restrict__ tw, int t) {
  Codelet<T, 8>::run(r, nullptr);
#pragma unroll
  for (int a = 1; a < 8; ++a) r[a] = r[a] * tw[(a - 1) * 4 + t];
  // element (a, t) at 4 a + t; lane L reads a = 2L (registers 0..3) and
  // 2L + 1 (registers 4..7)
  cpx<T>* w1 = buf + t;
#pragma unroll
  for (int a = 0; a < 8; ++a) w1[4 * a] = r[a];
  wave_sync();
  const cpx<T>* r1 = buf + 8 * t;
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = r1[i];
  wave_sync();
  dft4_reg(r[0], r[1], r[2], r[3]);
  dft4_reg(r[4], r[5], r[6], r[7]);
  // X[2L + 8 b] and X[2L + 1 + 8 b] into natural order, then X[t + 4 m]
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    buf[xw_nat(2 * t + 8 * b)] = r[b];
    buf[xw_nat(2 * t + 1 + 8 * b)] = r[4 + b];
  }
  wave_sync();
#pragma unroll
  for (int m = 0; m < 8; ++m) r[m] = buf[xw_nat(t + 4 * m)];
  wave_sync();
}

template <typename T, int N>
__device__ __forceinline__ void wave_fft(cpx<T> (&r)[8], cpx<T>* __restrict__ buf,
                                         const cpx<T>* __restrict__ tw, int t) {
  if constexpr (N == 512)
    wave_fft512<T>(r, buf, tw, t);
  else if constexpr (N == 256)
    wave_fft256<T>(r, buf, tw, t);
  else if constexpr (N == 192)
    wave_fft192<T>(r, buf, tw, t);
  else if constexpr (N == 128)
    wave_fft128<T>(r, buf, tw, t);
  else if constexpr (N == 96)
    wave_fft96<T>(r, buf, tw, t);
  else if constexpr (N == 64)
    wave_fft64<T>(r, buf, tw, t);
  else
    wave_fft32<T>(r, buf, tw, t);
}

// Forward transform of two finished real fields (b: none when !two), unpacked
// into the r2c spectra of rows `row` of fields fa and fa + 1; nothing is
// stored for a row past the end (valid false).
template <typename T, int N>
__device__ __forceinline__ void xw_forward(cpx<T> (&z)[8], cpx<T>* __restrict__ buf,
                                           const cpx<T>* __restrict__ tw, int t,
                                           cpx<T>* __restrict__ nl, long long fs, long long row,
                                           int nkxp, int fa, bool two, bool valid) {
  constexpr int S = N / 8, SN = S + S / 8;  // SN: natural-order slots per register
  wave_fft<T, N>(z, buf, tw, t);
  // slot of element t + S m (S a multiple of 8: a fixed step per register)
  const int t0 = xw_nat(t);
  auto slot = [&](int m) { return S % 8 == 0 ? t0 + SN * m : xw_nat(t + S * m); };
#pragma unroll
  for (int m = 0; m < 8; ++m) buf[slot(m)] = z[m];
  wave_sync();
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const int k = t + S * m;
    if (k <= N / 2 && valid) {
      const cpx<T> Zk = buf[slot(m)];
      const cpx<T> Zm = conj(buf[xw_nat(k == 0 ? 0 : N - k)]);
      nl[fa * fs + row * nkxp + k] = (Zk + Zm) * T(0.5);
      if (two) nl[(fa + 1) * fs + row * nkxp + k] = mul_mi(Zk - Zm) * T(0.5);
    }
  }
  wave_sync();
}

// Input addressing of the wave-level x pass: element kk of (kx, y) row `row`
// (plane row / ny) at rb + xo, with rb per row and xo per register; row-major
// rows (stride nkxp) or the blocked layout of the y pass (the 4 kx columns of
// a block contiguous over y, blocks ny * 4 apart).
__device__ __forceinline__ long long xw_row_base(long long row, int ny, int nkxp, bool blk) {
  if (!blk) return row * nkxp;
  const long long pl = row / ny;
  return pl * ny * nkxp + (row - pl * ny) * 4;
}
__device__ __forceinline__ int xw_col_off(int kk, int ny, bool blk) {
  return blk ? (kk >> 2) * ny * 4 + (kk & 3) : kk;
}

// NL_f = -(u dq_f/dx + v dq_f/dy + w dq_f/dz) on rows of N points.
// The generic schedule: real quantities in the order u, v, w, then per field
// dq/dx, dq/dy, dq/dz, consecutive pairs sharing one inverse transform (the
// value slots are read twice), and the forward transform of a pair of
// finished fields as soon as both are complete.  Used for three fields at
// 512 points, where the one-read schedule below needs more registers than
// two waves per SIMD allow, and at 192, where it spills more (three fields
// elsewhere: the one-read schedule, 7% faster at 256 and 9% at 128).
template <typename T, int NF, int N, bool BLK>
__global__ __launch_bounds__(64 * XW_WAVES, (N == 192 || N == 96 || N == 32) ? 2 : 1) void k_x_nlw_q(XArgs a, const cpx<T>* __restrict__ xyb,
                                                           cpx<T>* __restrict__ nl, long long fs,
                                                           long long nrows) {
  constexpr int NQ = 3 + 3 * NF, NP = (NQ + 1) / 2;
  constexpr int S = N / 8, RPW = 64 / S;  // lanes per row, rows per wave
  __shared__ cpx<T> tw[XW_TW];
  __shared__ cpx<T> xbuf[XW_WAVES][XW_BUF];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  xw_twiddles<T, N>(tw, tid);
  __syncthreads();
  // the 64 mod S spare lanes (192, 96) repeat the last lanes of row RPW - 1
  const bool spare = lane >= S * RPW;
  const int ln = spare ? lane - S : lane;
  const int t = ln % S, half = ln / S;
  cpx<T>* buf = xbuf[wv] + half * (XW_BUF / RPW);
  const int nkxp = a.nkxp;
  const T kxs = (T)a.kxs;
  const T sc = T(1) / T(N);
  // input offsets per register: kk itself (row-major, folded into the
  // loads) or its place in the blocked layout
  constexpr bool blk = BLK;
  int xo[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int k = t + S * m;
    xo[m] = xw_col_off(k <= N / 2 ? k : N - k, a.ny, blk);
  }
  for (long long rw = (long long)blockIdx.x * XW_WAVES + wv; rw * RPW < nrows;
       rw += (long long)gridDim.x * XW_WAVES) {
    // a row past the end (in the last wave) computes on a copy of the last
    // row and stores nothing; spare lanes compute what their twin lanes do
    const long long row0 = rw * RPW + half;
    const bool inr = RPW == 1 || row0 < nrows;
    const bool valid = inr && !spare;
    const long long row = inr ? row0 : nrows - 1;
    T U[3][8];
    T acc[NF][8];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      // keep each pair's loads next to its transform (hoisting them all would
      // multiply the live registers)
      __builtin_amdgcn_sched_barrier(0);
      // the two quantities of this pair (qb = NQ: none)
      const int qa = 2 * p, qb = 2 * p + 1;
      cpx<T> r[8];
      const long long rb = xw_row_base(row, a.ny, nkxp, blk);
      auto src = [&](int q, bool& dx) -> const cpx<T>* {
        dx = false;
        if (q < 3) return xyb + (3 * q) * fs + rb;
        const int f = (q - 3) / 3, d = (q - 3) % 3;
        dx = d == 0;
        return xyb + (3 * f + d) * fs + rb;
      };
      bool dxa, dxb = false;
      const cpx<T>* pa = src(qa, dxa);
      const cpx<T>* pb = qb < NQ ? src(qb, dxb) : nullptr;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int k = t + S * m;
        const int kk = k <= N / 2 ? k : N - k;
        cpx<T> A = pa[xo[m]];
        cpx<T> B = pb ? pb[xo[m]] : zero<T>();
        const T kx = (kk == N / 2) ? T(0) : kxs * (T)kk;
        if (dxa) A = mul_i(A) * kx;
        if (dxb) B = mul_i(B) * kx;
        if (kk == 0 || kk == N / 2) {
          A.y = T(0);
          B.y = T(0);
        }
        // Z[k] = A + i B (k <= N/2), conj(A) + i conj(B) (k > N/2); inverse via conj
        const cpx<T> Z = (k <= N / 2) ? mk(A.x - B.y, A.y + B.x) : mk(A.x + B.y, B.x - A.y);
        r[m] = conj(Z);
      }
      wave_fft<T, N>(r, buf, tw, t);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = 2 * p + h;
        if (q >= NQ) continue;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const T val = h == 0 ? r[m].x * sc : -r[m].y * sc;
          if (q < 3) {
            U[q][m] = val;
          } else {
            const int f = (q - 3) / 3, d = (q - 3) % 3;
            if (d == 0)
              acc[f][m] = -U[0][m] * val;
            else
              acc[f][m] -= U[d][m] * val;
          }
        }
        // a pair of fields finished: forward transform and unpack
        if (q >= 3 && (q - 3) % 3 == 2) {
          const int f = (q - 3) / 3;
          if (f % 2 == 1 || f == NF - 1) {
            const int fa = f % 2 == 1 ? f - 1 : f;
            const bool two = f % 2 == 1;
            cpx<T> z[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) z[m] = mk(acc[fa][m], two ? acc[fa + 1][m] : T(0));
            xw_forward<T, N>(z, buf, tw, t, nl, fs, row, nkxp, fa, two, valid);
          }
        }
      }
    }
  }
}

// (two waves per SIMD asked for explicitly at N = 192, 128 and 96, where the
// compiler would otherwise go past 256 registers)
template <typename T, int NF, int N, bool BLK>
__global__ __launch_bounds__(64 * XW_WAVES, (N == 192 || N == 128 || N == 96) ? 2 : 1) void k_x_nlw(XArgs a, const cpx<T>* __restrict__ xyb,
                                                         cpx<T>* __restrict__ nl, long long fs,
                                                         long long nrows) {
  // Three or four fields: pairs of real quantities per complex transform,
  // each spectral slot read once: (u, du/dx), (v, dv/dx), (w, dw/dx) from
  // one load each (the x derivative is i k~x times the same coefficients),
  // then (dq_f/dy, dq_f/dz) for f = 0..2, and for theta (dq/dx, dq/dy), (dq/dz).
  // NL_f = -(u dq_f/dx + v dq_f/dy + w dq_f/dz) accumulates in that order
  // as soon as u is known; each pair of finished fields is transformed
  // forward together.
  static_assert(NF == 3 || NF == 4, "three or four fields");
  constexpr int NP = NF == 4 ? 8 : 6;
  constexpr int TH = NF - 1;  // theta's accumulator (four fields)
  constexpr int S = N / 8, RPW = 64 / S;  // lanes per row, rows per wave
  __shared__ cpx<T> tw[XW_TW];
  __shared__ cpx<T> xbuf[XW_WAVES][XW_BUF];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  xw_twiddles<T, N>(tw, tid);
  __syncthreads();
  // the 64 mod S spare lanes (192, 96) repeat the last lanes of row RPW - 1
  const bool spare = lane >= S * RPW;
  const int ln = spare ? lane - S : lane;
  const int t = ln % S, half = ln / S;
  cpx<T>* buf = xbuf[wv] + half * (XW_BUF / RPW);
  const int nkxp = a.nkxp;
  const T kxs = (T)a.kxs;
  const T sc = T(1) / T(N);
  // input offsets per register: kk itself (row-major, folded into the
  // loads) or its place in the blocked layout
  constexpr bool blk = BLK;
  int xo[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int k = t + S * m;
    xo[m] = xw_col_off(k <= N / 2 ? k : N - k, a.ny, blk);
  }
  for (long long rw = (long long)blockIdx.x * XW_WAVES + wv; rw * RPW < nrows;
       rw += (long long)gridDim.x * XW_WAVES) {
    // a row past the end (in the last wave) computes on a copy of the last
    // row and stores nothing; spare lanes compute what their twin lanes do
    const long long row0 = rw * RPW + half;
    const bool inr = RPW == 1 || row0 < nrows;
    const bool valid = inr && !spare;
    const long long row = inr ? row0 : nrows - 1;
    T U[3][8];
    T acc[NF][8];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      // keep each pair's loads next to its transform (hoisting them all would
      // multiply the live registers)
      __builtin_amdgcn_sched_barrier(0);
      // slot of A; B: the x derivative of A (p < 3), another slot, or none
      const int slotA = p < 3 ? 3 * p : p < 6 ? 3 * (p - 3) + 1 : (p == 6 ? 9 : 11);
      const bool dxA = p == 6;
      const bool sameB = p < 3;
      const bool hasB = p < 7;
      const int slotB = p < 3 ? slotA : p < 6 ? 3 * (p - 3) + 2 : 10;
      const long long rb = xw_row_base(row, a.ny, nkxp, blk);
      const cpx<T>* pa = xyb + slotA * fs + rb;
      const cpx<T>* pb = xyb + slotB * fs + rb;
      cpx<T> r[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int k = t + S * m;
        const int kk = k <= N / 2 ? k : N - k;
        const T kx = (kk == N / 2) ? T(0) : kxs * (T)kk;
        cpx<T> A = pa[xo[m]];
        cpx<T> B = sameB ? mul_i(A) * kx : (hasB ? pb[xo[m]] : zero<T>());
        if (dxA) A = mul_i(A) * kx;
        if (kk == 0 || kk == N / 2) {
          A.y = T(0);
          B.y = T(0);
        }
        // Z[k] = A + i B (k <= N/2), conj(A) + i conj(B) (k > N/2); inverse via conj
        const cpx<T> Z = (k <= N / 2) ? mk(A.x - B.y, A.y + B.x) : mk(A.x + B.y, B.x - A.y);
        r[m] = conj(Z);
      }
      wave_fft<T, N>(r, buf, tw, t);
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const T va = r[m].x * sc, vb = -r[m].y * sc;
        if (p < 3) {
          U[p][m] = va;
          acc[p][m] = -U[0][m] * vb;        // -u dq_p/dx (U[0] set by pair 0)
        } else if (p < 6) {
          acc[p - 3][m] -= U[1][m] * va;    // -v dq/dy
          acc[p - 3][m] -= U[2][m] * vb;    // -w dq/dz
        } else if (p == 6) {
          acc[TH][m] = -U[0][m] * va;
          acc[TH][m] -= U[1][m] * vb;
        } else {
          acc[TH][m] -= U[2][m] * va;
        }
      }
      if (p == 4) {
        cpx<T> z[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) z[m] = mk(acc[0][m], acc[1][m]);
        xw_forward<T, N>(z, buf, tw, t, nl, fs, row, nkxp, 0, true, valid);
      }
      if (p == NP - 1) {
        // the last field(s): 2 and theta together, or 2 alone
        cpx<T> z[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) z[m] = mk(acc[2][m], NF == 4 ? acc[TH][m] : T(0));
        xw_forward<T, N>(z, buf, tw, t, nl, fs, row, nkxp, 2, NF == 4, valid);
      }
    }
    // (the next row's loads stay behind this row's last transform)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ---------------------------------------------------------------- helpers
__global__ void k_fill(cpx<double>* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = zero<double>();
}

// Remove the physical mean of a mixed-space field: the (0,0) pencil holds
// sum_xy at every z, so subtract its z-average from every z.
__global__ void k_sub_mean00(cpx<double>* pmix, long long npen, int nz) {
  __shared__ double part[256];
  double s = 0.0;
  for (int z = threadIdx.x; z < nz; z += blockDim.x) s += pmix[(long long)z * npen].x;
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
    part[0] = t / nz;
  }
  __syncthreads();
  const double m = part[0];
  for (int z = threadIdx.x; z < nz; z += blockDim.x) pmix[(long long)z * npen].x -= m;
}

// ---------------------------------------------------------------- launchers
template <typename T>
void launch_y(const YArgs& a, bool big, bool inv, int mode, const cpx<T>* src, cpx<T>* dst,
              cpx<T>* dst2, long long sfs, long long dfs, int nplanes, int nfields,
              hipStream_t st) {
  const int L = (a.lines == 8 && y_wide_tiles(a)) ? 8 : YL;
  const long long nlines = (long long)nplanes * a.nkxp;
  const long long ntiles = (nlines + L - 1) / L;
  const long long yg = a.grid > 0 ? a.grid : Y_GRID;
  // fewer tiles than the persistent grid: one workgroup per tile, rounded up
  // to whole chunks of 64 so that the XCD-aware order still applies
  long long gx = ntiles < yg ? ntiles : yg;
  if (gx < yg && gx % 64) gx = std::min(yg, (gx + 63) / 64 * 64);
  dim3 grid((unsigned)gx, nfields);
  const size_t sh = y_lds_bytes(a.ny, a.pl.tsize, sizeof(cpx<T>), L);
  const int need = (a.ny + YNT / YL - 1) / (YNT / YL);
  const int iv = inv ? 1 : 0;
#define FCNS_YL(FPV, OWNV, LV)                                                                \
  do {                                                                                      \
    if (a.noprefetch)                                                                       \
      FCNS_LAUNCH((k_y<T, FPV, OWNV, false, LV>), grid, dim3(64 * LV), sh, st, a, src, dst,   \
                  dst2, sfs, dfs, nlines, iv, mode);                                        \
    else                                                                                    \
      FCNS_LAUNCH((k_y<T, FPV, OWNV, true, LV>), grid, dim3(64 * LV), sh, st, a, src, dst,    \
                  dst2, sfs, dfs, nlines, iv, mode);                                        \
  } while (0)
#define FCNS_Y(FPV, OWNV) FCNS_YL(FPV, OWNV, YL)
  if (y_wide_tiles(a)) {
    using P512 = SPlan<8, 8, 8>;
    if (L == 8)
      FCNS_YL(P512, 8, 8);
    else
      FCNS_Y(P512, 8);
  } else if (a.ny == 256 && plan_is(a.pl, {8, 8, 4})) {
    using P256 = SPlan<8, 8, 4>;
    FCNS_Y(P256, 4);
  } else if (a.ny == 192 && plan_is(a.pl, {8, 8, 3})) {
    using P192 = SPlan<8, 8, 3>;
    FCNS_Y(P192, 4);
  } else if (a.ny == 128 && plan_is(a.pl, {8, 8, 2})) {
    using P128 = SPlan<8, 8, 2>;
    FCNS_Y(P128, 4);
  } else if (a.ny == 96 && plan_is(a.pl, {8, 4, 3})) {
    using P96 = SPlan<8, 4, 3>;
    FCNS_Y(P96, 4);
  } else if (a.ny == 64 && plan_is(a.pl, {8, 8})) {
    using P64 = SPlan<8, 8>;
    FCNS_Y(P64, 4);
  } else if (big) {
    if (need <= 4) FCNS_Y(DynPlan<true>, 4); else if (need <= 8) FCNS_Y(DynPlan<true>, 8); else FCNS_Y(DynPlan<true>, 16);
  } else {
    if (need <= 4) FCNS_Y(DynPlan<false>, 4); else if (need <= 8) FCNS_Y(DynPlan<false>, 8); else FCNS_Y(DynPlan<false>, 16);
  }
#undef FCNS_Y
#undef FCNS_YL
}
template void launch_y<double>(const YArgs&, bool, bool, int, const cpx<double>*, cpx<double>*,
                               cpx<double>*, long long, long long, int, int, hipStream_t);
template void launch_y<float>(const YArgs&, bool, bool, int, const cpx<float>*, cpx<float>*,
                              cpx<float>*, long long, long long, int, int, hipStream_t);

void launch_x_r2c(const XArgs& a, bool big, const double* phys, cpx<double>* xy, long long pfs,
                  long long xfs, long long nrows, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((nrows + XR - 1) / XR), nfields);
  const size_t sh = ((size_t)a.pl.tsize + 2 * XL * x_ls(a.nx)) * sizeof(cpx<double>);
  if (big)
    FCNS_LAUNCH((k_x_r2c<double, true>), grid, dim3(XNT), sh, st, a, phys, xy, pfs, xfs, nrows);
  else
    FCNS_LAUNCH((k_x_r2c<double, false>), grid, dim3(XNT), sh, st, a, phys, xy, pfs, xfs, nrows);
}

void launch_x_c2r(const XArgs& a, bool big, const cpx<double>* xy, double* phys, long long xfs,
                  long long pfs, long long nrows, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((nrows + XR - 1) / XR), nfields);
  const size_t sh = ((size_t)a.pl.tsize + 2 * XL * x_ls(a.nx)) * sizeof(cpx<double>);
  if (big)
    FCNS_LAUNCH((k_x_c2r<double, true>), grid, dim3(XNT), sh, st, a, xy, phys, xfs, pfs, nrows);
  else
    FCNS_LAUNCH((k_x_c2r<double, false>), grid, dim3(XNT), sh, st, a, xy, phys, xfs, pfs, nrows);
}

template <typename T, class FP, int RR, int NT, int CC>
static void launch_x_nl_v(const XArgs& a, const cpx<T>* xyb, cpx<T>* nl, long long fs,
                          long long nrows, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((nrows + RR - 1) / RR));
  const size_t sh = ((size_t)a.pl.tsize + 2 * (RR / 2) * x_ls(a.nx)) * sizeof(cpx<T>);
  FCNS_LAUNCH((k_x_nl<T, FP, RR, NT, CC>), grid, dim3(NT), sh, st, a, xyb, nl, fs, nrows,
              nfields);
}

static bool x_wave_rows(int nx) {
  return nx == 512 || nx == 256 || nx == 192 || nx == 128 || nx == 96 || nx == 64 ||
         nx == 32;
}

bool x_reads_blocked(const XArgs& a) { return x_wave_rows(a.nx) && a.variant == 0; }

// nx = 512, 256, 192, 128, 96, 64 and 32: wave-level rows (variant 0) or the tiled kernels; other
// nx: 4 rows x 256 threads (variant 0, 1) or 8 rows x 512 threads (variant 2),
// with compile-time plans for 512 and 256; nx <= 256: 8 rows x nx threads
// (variant 3)
template <typename T>
void launch_x_nl(const XArgs& a, bool big, const cpx<T>* xyb, cpx<T>* nl, long long fs,
                 long long nrows, int nfields, hipStream_t st) {
  if (a.variant == 3 && a.nx <= 256) {
    // short rows: 8 rows (4 complex lines) per workgroup and one thread per
    // column (a radix-8 stage keeps half the threads busy; 4 or 16 rows, or
    // 4 rows over 256 threads, measured slower)
    const int nt = (a.nx + 63) / 64 * 64;
#define FCNS_XS(NTV)                                                                        \
  do {                                                                                      \
    if (big)                                                                                \
      launch_x_nl_v<T, DynPlan<true>, 8, NTV, 1>(a, xyb, nl, fs, nrows, nfields, st);       \
    else                                                                                    \
      launch_x_nl_v<T, DynPlan<false>, 8, NTV, 1>(a, xyb, nl, fs, nrows, nfields, st);      \
  } while (0)
    if (nt == 64)
      FCNS_XS(64);
    else if (nt == 128)
      FCNS_XS(128);
    else if (nt == 192)
      FCNS_XS(192);
    else
      FCNS_XS(256);
#undef FCNS_XS
  } else if (a.variant == 2 && a.nx <= 512) {
    if (a.nx == 512 && plan_is(a.pl, {8, 8, 8}))
      launch_x_nl_v<T, SPlan<8, 8, 8>, 8, 512, 1>(a, xyb, nl, fs, nrows, nfields, st);
    else if (big)
      launch_x_nl_v<T, DynPlan<true>, 8, 512, 1>(a, xyb, nl, fs, nrows, nfields, st);
    else
      launch_x_nl_v<T, DynPlan<false>, 8, 512, 1>(a, xyb, nl, fs, nrows, nfields, st);
  } else if (x_wave_rows(a.nx) && a.variant == 0) {
    // wave-level rows; enough workgroups to fill the chip several times
    const long long rpw = 64 / (a.nx / 8);
    const long long need = (nrows + rpw * XW_WAVES - 1) / (rpw * XW_WAVES);
    dim3 grid((unsigned)(need < 4096 ? need : 4096));
#define FCNS_XW(K, NFV, NV)                                                                  \
  do {                                                                                      \
    if (a.blk_in)                                                                           \
      FCNS_LAUNCH((K<T, NFV, NV, true>), grid, dim3(64 * XW_WAVES), 0, st, a, xyb, nl, fs,   \
                  nrows);                                                                   \
    else                                                                                    \
      FCNS_LAUNCH((K<T, NFV, NV, false>), grid, dim3(64 * XW_WAVES), 0, st, a, xyb, nl, fs,  \
                  nrows);                                                                   \
  } while (0)
    if (a.nx == 512 && nfields == 4)
      FCNS_XW(k_x_nlw, 4, 512);
    else if (a.nx == 512)
      FCNS_XW(k_x_nlw_q, 3, 512);
    else if (a.nx == 256 && nfields == 4)
      FCNS_XW(k_x_nlw, 4, 256);
    else if (a.nx == 256)
      FCNS_XW(k_x_nlw, 3, 256);
    else if (a.nx == 192 && nfields == 4)
      FCNS_XW(k_x_nlw, 4, 192);
    else if (a.nx == 192)
      FCNS_XW(k_x_nlw_q, 3, 192);
    else if (a.nx == 128 && nfields == 4)
      FCNS_XW(k_x_nlw, 4, 128);
    else if (a.nx == 128)
      FCNS_XW(k_x_nlw, 3, 128);
    else if (a.nx == 96 && nfields == 4)
      FCNS_XW(k_x_nlw, 4, 96);
    else if (a.nx == 96)
      FCNS_XW(k_x_nlw, 3, 96);
    else if (a.nx == 64 && nfields == 4)
      FCNS_XW(k_x_nlw, 4, 64);
    else if (a.nx == 64)
      FCNS_XW(k_x_nlw, 3, 64);
    else if (nfields == 4)
      FCNS_XW(k_x_nlw, 4, 32);
    else
      FCNS_XW(k_x_nlw, 3, 32);
#undef FCNS_XW
  } else if (a.nx == 512 && plan_is(a.pl, {8, 8, 8}))
    launch_x_nl_v<T, SPlan<8, 8, 8>, 4, 256, 2>(a, xyb, nl, fs, nrows, nfields, st);
  else if (a.nx == 256 && plan_is(a.pl, {8, 8, 4}))
    launch_x_nl_v<T, SPlan<8, 8, 4>, 4, 256, 1>(a, xyb, nl, fs, nrows, nfields, st);
  else if (big)
    launch_x_nl_v<T, DynPlan<true>, 4, 256, 2>(a, xyb, nl, fs, nrows, nfields, st);
  else
    launch_x_nl_v<T, DynPlan<false>, 4, 256, 2>(a, xyb, nl, fs, nrows, nfields, st);
}
template void launch_x_nl<double>(const XArgs&, bool, const cpx<double>*, cpx<double>*, long long,
                                  long long, int, hipStream_t);
template void launch_x_nl<float>(const XArgs&, bool, const cpx<float>*, cpx<float>*, long long,
                                 long long, int, hipStream_t);

void launch_fill(cpx<double>* p, long long n, hipStream_t st) {
  const int nt = 256;
  FCNS_LAUNCH(k_fill, dim3((unsigned)((n + nt - 1) / nt)), dim3(nt), 0, st, p, n);
}

void launch_sub_mean00(cpx<double>* pmix, long long npen, int nz, double, hipStream_t st) {
  FCNS_LAUNCH(k_sub_mean00, dim3(1), dim3(256), 0, st, pmix, npen, nz);
}

}  // namespace fcns
