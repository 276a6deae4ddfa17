// Periodic-direction kernels: FFTs along y (c2c) and x (r2c / c2r), and the
// fused x-pass that evaluates the advective products in physical space.
//
// Layouts (x fastest): physical real fields [planes][ny][nx]; (kx, y) and
// (kx, ky) complex fields [planes][ny][nkxp] holding nkx = nx/2 + 1 modes per
// row, the row stride nkxp padded to a multiple of 4 (64 B).  Inverse
// transforms use IFFT(y) = conj(FFT(conj(y))) / n with the conjugations folded
// into loads and stores.
#include "kernels.hpp"

namespace fcns {

// ---------------------------------------------------------------- y pass
// Lines q = plane * nkxp + kx; a tile is YL consecutive lines, staged in LDS
// interleaved (element ky of line l at lds_pos<true>(l, ky, YL, 1), y_span
// slots per buffer).  Each thread keeps one line of the tile (l = tid % YL,
// YNT being a multiple of YL) and the rows ky = tid / YL + r * YNT / YL.
// Workgroups loop over tiles and load the next tile into registers before
// transforming the current one, so the loads overlap the FFT.  mode 1
// (inverse only): a second pass transforms i k~y times the input into dst2.
__host__ __device__ inline int y_span(int ny) { return YL * (ny + ny / 8 + 1); }

size_t y_lds_bytes(int ny, int tsize, size_t elem) {
  return ((size_t)tsize + 2 * (size_t)y_span(ny)) * elem;
}

template <typename T, class FP, int OWN>
__global__ __launch_bounds__(YNT) void k_y(YArgs a, const cpx<T>* src, cpx<T>* dst, cpx<T>* dst2,
                                           long long sfs, long long dfs, long long nlines, int inv,
                                           int mode) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int ny = FP::dynamic ? a.ny : FP::n;
  const int nkx = a.nkx, nkxp = a.nkxp;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + a.pl.tsize;
  cpx<T>* X1 = X0 + y_span(ny);
  src += blockIdx.y * sfs;
  dst += blockIdx.y * dfs;
  if (mode == 1) dst2 += blockIdx.y * dfs;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < a.pl.tsize; i += YNT) tw[i] = gtw[i];
  const int l = tid % YL, ky0 = tid / YL;
  constexpr int KYS = YNT / YL;
  const long long ntiles = (nlines + YL - 1) / YL;
  const T sc = inv ? T(1) / (T)ny : T(1);
  const int npass = (mode == 1) ? 2 : 1;
  cpx<T> cur[OWN], nxt[OWN];
  long long t = blockIdx.x;
  auto line_base = [&](long long tt, bool& ok) {
    const long long q = tt * YL + l;
    const long long pl = q / nkxp, kx = q - pl * nkxp;
    ok = q < nlines && kx < nkx;
    return ok ? pl * ny * nkxp + kx : 0;  // element ky at base + ky * nkxp
  };
  {
    bool ok;
    const long long base = line_base(t, ok);
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int ky = ky0 + r * KYS;
      cur[r] = (ok && ky < ny) ? src[base + (long long)ky * nkxp] : zero<T>();
    }
  }
  for (; t < ntiles; t += gridDim.x) {
    bool ok, okn;
    const long long base = line_base(t, ok);
    const long long tn = t + gridDim.x;
    const long long basen = line_base(tn, okn);
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int ky = ky0 + r * KYS;
      nxt[r] = (okn && ky < ny) ? src[basen + (long long)ky * nkxp] : zero<T>();
    }
    for (int pass = 0; pass < npass; ++pass) {
#pragma unroll
      for (int r = 0; r < OWN; ++r) {
        const int ky = ky0 + r * KYS;
        if (ky < ny) {
          cpx<T> v = cur[r];
          if (pass == 1) v = mul_i(v) * (T)k_odd(ky, ny, a.kys);
          X0[lds_pos<true>(l, ky, YL, 1)] = inv ? conj(v) : v;
        }
      }
      __syncthreads();
      const cpx<T>* R = fft_run<T, YL, YNT, true, FP>(X0, X1, YL, 1, a.pl, tw, tid);
      cpx<T>* out = pass ? dst2 : dst;
      if (ok) {
#pragma unroll
        for (int r = 0; r < OWN; ++r) {
          const int ky = ky0 + r * KYS;
          if (ky < ny) {
            const cpx<T> v = R[lds_pos<true>(l, ky, YL, 1)];
            out[base + (long long)ky * nkxp] = (inv ? conj(v) : v) * sc;
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < OWN; ++r) cur[r] = nxt[r];
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
  const long long nlines = (long long)nplanes * a.nkxp;
  const long long ntiles = (nlines + YL - 1) / YL;
  dim3 grid((unsigned)(ntiles < Y_GRID ? ntiles : Y_GRID), nfields);
  const size_t sh = y_lds_bytes(a.ny, a.pl.tsize, sizeof(cpx<T>));
  const int need = (a.ny + YNT / YL - 1) / (YNT / YL);
  const int iv = inv ? 1 : 0;
#define FCNS_Y(FPV, OWNV)                                                                    \
  FCNS_LAUNCH((k_y<T, FPV, OWNV>), grid, dim3(YNT), sh, st, a, src, dst, dst2, sfs, \
                     dfs, nlines, iv, mode)
  if (a.ny == 512 && plan_is(a.pl, {8, 8, 8})) {
    using P512 = SPlan<8, 8, 8>;
    FCNS_Y(P512, 8);
  } else if (a.ny == 256 && plan_is(a.pl, {8, 8, 4})) {
    using P256 = SPlan<8, 8, 4>;
    FCNS_Y(P256, 4);
  } else if (big) {
    if (need <= 4) FCNS_Y(DynPlan<true>, 4); else if (need <= 8) FCNS_Y(DynPlan<true>, 8); else FCNS_Y(DynPlan<true>, 16);
  } else {
    if (need <= 4) FCNS_Y(DynPlan<false>, 4); else if (need <= 8) FCNS_Y(DynPlan<false>, 8); else FCNS_Y(DynPlan<false>, 16);
  }
#undef FCNS_Y
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

// 4 rows x 256 threads; compile-time plans for nx = 512 and 256
template <typename T>
void launch_x_nl(const XArgs& a, bool big, const cpx<T>* xyb, cpx<T>* nl, long long fs,
                 long long nrows, int nfields, hipStream_t st) {
  if (a.nx == 512 && plan_is(a.pl, {8, 8, 8}))
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
