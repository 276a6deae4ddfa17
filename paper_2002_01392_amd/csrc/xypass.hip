// Periodic-direction kernels: FFTs along y (c2c) and x (r2c / c2r), and the
// fused x-pass that evaluates the advective products in physical space.
//
// Layouts (x fastest): physical real fields [planes][ny][nx]; (kx, y) and
// (kx, ky) complex fields [planes][ny][nkx], nkx = nx/2 + 1.  Inverse
// transforms use IFFT(y) = conj(FFT(conj(y))) / n with the conjugations folded
// into loads and stores.
#include "kernels.hpp"

namespace fcns {

// ---------------------------------------------------------------- y pass
// Lines q = plane * nkx + kx; a workgroup takes YL consecutive lines, staged
// in LDS as X[ky * YL + l].  mode 1 (inverse only): a second pass transforms
// i k~y times the input into dst2.
template <typename T, bool BIG, int OWN>
__global__ __launch_bounds__(YNT) void k_y(YArgs a, const cpx<double>* src, cpx<double>* dst,
                                           cpx<double>* dst2, long long sfs, long long dfs,
                                           long long nlines, int inv, int mode) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int ny = a.ny, nkx = a.nkx;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + ny;
  cpx<T>* X1 = X0 + ny * YL;
  src += blockIdx.y * sfs;
  dst += blockIdx.y * dfs;
  if (mode == 1) dst2 += blockIdx.y * dfs;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < ny; i += YNT) tw[i] = gtw[i];
  const long long q0 = (long long)blockIdx.x * YL;
  const int tot = ny * YL;
  cpx<double> keep[OWN];
#pragma unroll
  for (int r = 0; r < OWN; ++r) {
    const int e = tid + r * YNT;
    keep[r] = zero<double>();
    if (e < tot) {
      const int ky = e / YL;
      const long long q = q0 + e % YL;
      if (q < nlines) {
        const long long pl = q / nkx, kx = q - pl * nkx;
        keep[r] = src[(pl * ny + ky) * nkx + kx];
      }
    }
  }
  const double sc = inv ? 1.0 / ny : 1.0;
  const int npass = (mode == 1) ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int e = tid + r * YNT;
      if (e < tot) {
        cpx<double> v = keep[r];
        if (pass == 1) v = mul_i(v) * k_odd(e / YL, ny, a.kys);
        X0[e] = cvt<T>(inv ? conj(v) : v);
      }
    }
    __syncthreads();
    const cpx<T>* R = fft_fwd<T, YL, BIG>(X0, X1, YL, 1, a.pl, tw, tid, YNT);
    cpx<double>* out = pass ? dst2 : dst;
    for (int e = tid; e < tot; e += YNT) {
      const int ky = e / YL;
      const long long q = q0 + e % YL;
      if (q < nlines) {
        const long long pl = q / nkx, kx = q - pl * nkx;
        const cpx<double> v = cvt<double>(R[e]);
        out[(pl * ny + ky) * nkx + kx] = (inv ? conj(v) : v) * sc;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- x helpers
// Rows r0..r0+XR-1; two real rows (2a, 2a+1) share complex line a:
// z[n] = x_2a[n] + i x_2a+1[n], staged in LDS as X[n * XL + a].
constexpr int XL = XR / 2;

// Pack the spectra A (row 2a), B (row 2a+1) of two real rows into the
// conjugate of the full spectrum of z = x_2a + i x_2a+1 (ready for the inverse
// via the conjugated forward transform).  The imaginary parts of the kx = 0
// and kx = nx/2 bins are dropped, as a c2r transform does.  dx: multiply by
// i k~x first.
template <typename T>
__device__ __forceinline__ void x_pack_c2r(cpx<T>* X, const cpx<double>* __restrict__ xy,
                                           long long r0, long long nrows, const XArgs& a,
                                           bool dx, int tid) {
  const int nx = a.nx, nkx = a.nkx;
  for (int e = tid; e < XL * nkx; e += XNT) {
    const int al = e / nkx, k = e - al * nkx;
    const long long ra = r0 + 2 * al, rb = ra + 1;
    cpx<double> A = (ra < nrows) ? xy[ra * nkx + k] : zero<double>();
    cpx<double> B = (rb < nrows) ? xy[rb * nkx + k] : zero<double>();
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
    X[k * XL + al] = cvt<T>(conj(mk(A.x - B.y, A.y + B.x)));
    if (k > 0 && 2 * k < nx) X[(nx - k) * XL + al] = cvt<T>(conj(mk(A.x + B.y, B.x - A.y)));
  }
}

// Unpack the forward transform of two packed real rows into their r2c spectra.
template <typename T>
__device__ __forceinline__ void x_unpack_r2c(const cpx<T>* X, cpx<double>* __restrict__ xy,
                                             long long r0, long long nrows, const XArgs& a,
                                             int tid) {
  const int nx = a.nx, nkx = a.nkx;
  for (int e = tid; e < XL * nkx; e += XNT) {
    const int al = e / nkx, k = e - al * nkx;
    const cpx<double> Z = cvt<double>(X[k * XL + al]);
    const cpx<double> Zm = conj(cvt<double>(X[((nx - k) % nx) * XL + al]));
    const long long ra = r0 + 2 * al, rb = ra + 1;
    if (ra < nrows) xy[ra * nkx + k] = (Z + Zm) * 0.5;
    if (rb < nrows) xy[rb * nkx + k] = mul_mi(Z - Zm) * 0.5;
  }
}

// physical value of row rl, column n in an inverse-transformed packed buffer
// (conjugated forward output): real part for even rows, imaginary for odd
template <typename T>
__device__ __forceinline__ double x_phys(const cpx<T>* R, int rl, int n) {
  const cpx<T> z = R[n * XL + (rl >> 1)];
  return (rl & 1) ? -(double)z.y : (double)z.x;
}

// ---------------------------------------------------------------- x r2c / c2r
template <typename T, bool BIG>
__global__ __launch_bounds__(XNT) void k_x_r2c(XArgs a, const double* __restrict__ phys,
                                               cpx<double>* __restrict__ xy, long long pfs,
                                               long long xfs, long long nrows) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int nx = a.nx;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + nx;
  cpx<T>* X1 = X0 + nx * XL;
  phys += blockIdx.y * pfs;
  xy += blockIdx.y * xfs;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < nx; i += XNT) tw[i] = gtw[i];
  const long long r0 = (long long)blockIdx.x * XR;
  T* Xs = reinterpret_cast<T*>(X0);
  for (int e = tid; e < XR * nx; e += XNT) {
    const int rl = e / nx, n = e - rl * nx;
    const long long r = r0 + rl;
    Xs[2 * (n * XL + (rl >> 1)) + (rl & 1)] = (r < nrows) ? (T)phys[r * nx + n] : T(0);
  }
  __syncthreads();
  const cpx<T>* R = fft_fwd<T, XL, BIG>(X0, X1, XL, 1, a.pl, tw, tid, XNT);
  x_unpack_r2c<T>(R, xy, r0, nrows, a, tid);
}

template <typename T, bool BIG>
__global__ __launch_bounds__(XNT) void k_x_c2r(XArgs a, const cpx<double>* __restrict__ xy,
                                               double* __restrict__ phys, long long xfs,
                                               long long pfs, long long nrows) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int nx = a.nx;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + nx;
  cpx<T>* X1 = X0 + nx * XL;
  phys += blockIdx.y * pfs;
  xy += blockIdx.y * xfs;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < nx; i += XNT) tw[i] = gtw[i];
  const long long r0 = (long long)blockIdx.x * XR;
  x_pack_c2r<T>(X0, xy, r0, nrows, a, false, tid);
  __syncthreads();
  const cpx<T>* R = fft_fwd<T, XL, BIG>(X0, X1, XL, 1, a.pl, tw, tid, XNT);
  const double sc = 1.0 / nx;
  for (int e = tid; e < XR * nx; e += XNT) {
    const int rl = e / nx, n = e - rl * nx;
    const long long r = r0 + rl;
    if (r < nrows) phys[r * nx + n] = x_phys<T>(R, rl, n) * sc;
  }
}

// ---------------------------------------------------------------- x pass with products
// NL_f = -(u dq_f/dx + v dq_f/dy + w dq_f/dz) at the physical points of XR
// rows (Sec. 4.2: derivatives in Fourier space, products in real space, no
// padding), then its r2c transform.  Passes: 0-2 physical u, v, w; then per
// field f: dq/dx, dq/dy, dq/dz (inverse), and the forward transform of NL_f.
template <typename T, bool BIG, int OWN>
__global__ __launch_bounds__(XNT) void k_x_nl(XArgs a, const cpx<double>* __restrict__ xyb,
                                              cpx<double>* __restrict__ nl, long long fs,
                                              long long nrows, int nfields) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int nx = a.nx;
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem);
  cpx<T>* X0 = tw + nx;
  cpx<T>* X1 = X0 + nx * XL;
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < nx; i += XNT) tw[i] = gtw[i];
  const long long r0 = (long long)blockIdx.x * XR;
  const int tot = XR * nx;
  const double sc = 1.0 / nx;
  double U[3][OWN];
  double acc[OWN];
  const int npass = 3 + 4 * nfields;
  for (int pass = 0; pass < npass; ++pass) {
    // which transform: comp c (pass < 3), else field f and sub-pass k
    const int f = (pass - 3) >> 2, k = (pass - 3) & 3;
    const bool fwd = pass >= 3 && k == 3;
    if (!fwd) {
      const cpx<double>* src;
      bool dx = false;
      if (pass < 3) {
        src = xyb + (3 * pass) * fs;
      } else if (k == 0) {
        src = xyb + (3 * f) * fs;
        dx = true;
      } else {
        src = xyb + (3 * f + k) * fs;
      }
      x_pack_c2r<T>(X0, src, r0, nrows, a, dx, tid);
    } else {
      T* Xw = reinterpret_cast<T*>(X0);
#pragma unroll
      for (int r = 0; r < OWN; ++r) {
        const int e = tid + r * XNT;
        if (e < tot) {
          const int rl = e / nx, n = e - rl * nx;
          Xw[2 * (n * XL + (rl >> 1)) + (rl & 1)] = (T)acc[r];
        }
      }
    }
    __syncthreads();
    const cpx<T>* R = fft_fwd<T, XL, BIG>(X0, X1, XL, 1, a.pl, tw, tid, XNT);
    if (pass < 3) {
#pragma unroll
      for (int r = 0; r < OWN; ++r) {
        const int e = tid + r * XNT;
        const int rl = e / nx, n = e - rl * nx;
        const double v = (e < tot) ? x_phys<T>(R, rl, n) * sc : 0.0;
        if (pass == 0) U[0][r] = v;
        else if (pass == 1) U[1][r] = v;
        else U[2][r] = v;
      }
    } else if (!fwd) {
#pragma unroll
      for (int r = 0; r < OWN; ++r) {
        const int e = tid + r * XNT;
        const int rl = e / nx, n = e - rl * nx;
        const double d = (e < tot) ? x_phys<T>(R, rl, n) * sc : 0.0;
        const double u = (k == 0) ? U[0][r] : ((k == 1) ? U[1][r] : U[2][r]);
        if (k == 0) acc[r] = -u * d;
        else acc[r] -= u * d;
      }
    } else {
      x_unpack_r2c<T>(R, nl + f * fs, r0, nrows, a, tid);
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
void launch_y(const YArgs& a, bool big, bool inv, int mode, const cpx<double>* src,
              cpx<double>* dst, cpx<double>* dst2, long long sfs, long long dfs, int nplanes,
              int nfields, hipStream_t st) {
  const long long nlines = (long long)nplanes * a.nkx;
  dim3 grid((unsigned)((nlines + YL - 1) / YL), nfields);
  const size_t sh = (size_t)a.ny * (2 * YL + 1) * sizeof(cpx<double>);
  const int need = (a.ny * YL + YNT - 1) / YNT;
  const int iv = inv ? 1 : 0;
#define FCNS_Y(BIGV, OWNV)                                                                    \
  FCNS_LAUNCH((k_y<double, BIGV, OWNV>), grid, dim3(YNT), sh, st, a, src, dst, dst2, sfs, \
                     dfs, nlines, iv, mode)
  if (big) {
    if (need <= 4) FCNS_Y(true, 4); else if (need <= 8) FCNS_Y(true, 8); else FCNS_Y(true, 16);
  } else {
    if (need <= 4) FCNS_Y(false, 4); else if (need <= 8) FCNS_Y(false, 8); else FCNS_Y(false, 16);
  }
#undef FCNS_Y
}

void launch_x_r2c(const XArgs& a, bool big, const double* phys, cpx<double>* xy, long long pfs,
                  long long xfs, long long nrows, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((nrows + XR - 1) / XR), nfields);
  const size_t sh = (size_t)a.nx * (2 * XL + 1) * sizeof(cpx<double>);
  if (big)
    FCNS_LAUNCH((k_x_r2c<double, true>), grid, dim3(XNT), sh, st, a, phys, xy, pfs, xfs, nrows);
  else
    FCNS_LAUNCH((k_x_r2c<double, false>), grid, dim3(XNT), sh, st, a, phys, xy, pfs, xfs, nrows);
}

void launch_x_c2r(const XArgs& a, bool big, const cpx<double>* xy, double* phys, long long xfs,
                  long long pfs, long long nrows, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((nrows + XR - 1) / XR), nfields);
  const size_t sh = (size_t)a.nx * (2 * XL + 1) * sizeof(cpx<double>);
  if (big)
    FCNS_LAUNCH((k_x_c2r<double, true>), grid, dim3(XNT), sh, st, a, xy, phys, xfs, pfs, nrows);
  else
    FCNS_LAUNCH((k_x_c2r<double, false>), grid, dim3(XNT), sh, st, a, xy, phys, xfs, pfs, nrows);
}

void launch_x_nl(const XArgs& a, bool big, const cpx<double>* xyb, cpx<double>* nl,
                 long long fs, long long nrows, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((nrows + XR - 1) / XR));
  const size_t sh = (size_t)a.nx * (2 * XL + 1) * sizeof(cpx<double>);
  const int need = (XR * a.nx + XNT - 1) / XNT;
#define FCNS_X(BIGV, OWNV)                                                                    \
  FCNS_LAUNCH((k_x_nl<double, BIGV, OWNV>), grid, dim3(XNT), sh, st, a, xyb, nl, fs, nrows, \
                     nfields)
  if (big) {
    if (need <= 4) FCNS_X(true, 4); else if (need <= 8) FCNS_X(true, 8); else FCNS_X(true, 16);
  } else {
    if (need <= 4) FCNS_X(false, 4); else if (need <= 8) FCNS_X(false, 8); else FCNS_X(false, 16);
  }
#undef FCNS_X
}

void launch_fill(cpx<double>* p, long long n, hipStream_t st) {
  const int nt = 256;
  FCNS_LAUNCH(k_fill, dim3((unsigned)((n + nt - 1) / nt)), dim3(nt), 0, st, p, n);
}

void launch_sub_mean00(cpx<double>* pmix, long long npen, int nz, double, hipStream_t st) {
  FCNS_LAUNCH(k_sub_mean00, dim3(1), dim3(256), 0, st, pmix, npen, nz);
}

}  // namespace fcns
