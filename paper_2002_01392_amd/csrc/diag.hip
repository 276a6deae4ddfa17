// Flow diagnostics from the mixed (kx, ky, z) fields of the state, by Parseval:
// for a real field with r2c coefficients q^ (unnormalised), the x-y mean of
// q^2 at height z is sum_{ky, kx >= 0} w(kx) |q^|^2 / (nx ny)^2 with w = 1 at
// kx = 0 and kx = nx/2 and 2 in between.  One workgroup per z plane reduces
// |u^|^2, |v^|^2, |w^|^2, |theta^|^2 and |div^|^2 (div = i k~x u + i k~y v +
// dw/dz, the FC divergence of Sec. 6) in a fixed order, so the result is
// reproducible; the host adds the planes.
#include "kernels.hpp"

namespace fcns {

constexpr int DNT = 256;

// mv: slot 2f = q_f, slot 2f+1 = dq_f/dz (mixed, stride ms per slot)
__global__ __launch_bounds__(DNT) void k_diag_planes(Geom g, const cpx<double>* __restrict__ mv,
                                                     long long ms, int nf, double* __restrict__ out) {
  __shared__ double red[DNT][5];
  const int z = blockIdx.x, tid = threadIdx.x;
  const long long plane = (long long)z * g.npen;
  double acc[5] = {0, 0, 0, 0, 0};
  for (long long p = tid; p < g.npen; p += DNT) {
    const int iy = (int)(p / g.nkxp), ix = (int)(p - (long long)iy * g.nkxp);
    if (ix >= g.nkx) continue;
    const double wgt = (ix == 0 || 2 * ix == g.nx) ? 1.0 : 2.0;
    const cpx<double> u = mv[plane + p], v = mv[2 * ms + plane + p];
    const cpx<double> w = mv[4 * ms + plane + p], dw = mv[5 * ms + plane + p];
    const double kx = (2 * ix == g.nx) ? 0.0 : g.kxs * ix;
    const double ky = k_odd(iy, g.ny, g.kys);
    const cpx<double> dv = mul_i(u * kx + v * ky) + dw;
    acc[0] += wgt * (u.x * u.x + u.y * u.y);
    acc[1] += wgt * (v.x * v.x + v.y * v.y);
    acc[2] += wgt * (w.x * w.x + w.y * w.y);
    if (nf == 4) {
      const cpx<double> t = mv[6 * ms + plane + p];
      acc[3] += wgt * (t.x * t.x + t.y * t.y);
    }
    acc[4] += wgt * (dv.x * dv.x + dv.y * dv.y);
  }
  for (int q = 0; q < 5; ++q) red[tid][q] = acc[q];
  __syncthreads();
  for (int h = DNT / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int q = 0; q < 5; ++q) red[tid][q] += red[tid + h][q];
    __syncthreads();
  }
  if (tid < 5) out[z * 5 + tid] = red[0][tid];
}

// 1D spectra of one mixed field at height z (Sec. 6): ex[kx] = sum_ky w(kx)
// |q^|^2, ey[ky] = sum over all kx of |q^(kx, ky)|^2, the negative kx taken
// from the conjugate-symmetric half (|q^(-kx, ky)| = |q^(kx, -ky)|); both
// normalised by (nx ny)^2.
__global__ __launch_bounds__(DNT) void k_spectra(Geom g, const cpx<double>* __restrict__ q, int z,
                                                 double* __restrict__ ex, double* __restrict__ ey) {
  const long long plane = (long long)z * g.npen;
  const double nrm = 1.0 / ((double)g.nx * g.ny * (double)g.nx * g.ny);
  for (int ix = threadIdx.x; ix < g.nkx; ix += DNT) {
    const double wgt = (ix == 0 || 2 * ix == g.nx) ? 1.0 : 2.0;
    double s = 0.0;
    for (int iy = 0; iy < g.ny; ++iy) {
      const cpx<double> a = q[plane + (long long)iy * g.nkxp + ix];
      s += a.x * a.x + a.y * a.y;
    }
    ex[ix] = wgt * s * nrm;
  }
  for (int iy = threadIdx.x; iy < g.ny; iy += DNT) {
    const int jy = (g.ny - iy) % g.ny;
    double s = 0.0;
    for (int ix = 0; ix < g.nkx; ++ix) {
      const cpx<double> a = q[plane + (long long)iy * g.nkxp + ix];
      s += a.x * a.x + a.y * a.y;
      if (ix != 0 && 2 * ix != g.nx) {
        const cpx<double> b = q[plane + (long long)jy * g.nkxp + ix];
        s += b.x * b.x + b.y * b.y;
      }
    }
    ey[iy] = s * nrm;
  }
}

void launch_diag_planes(const Geom& g, const cpx<double>* mv, long long ms, int nf, double* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_diag_planes, dim3(g.nz), dim3(DNT), 0, st, g, mv, ms, nf, out);
}

void launch_spectra(const Geom& g, const cpx<double>* q, int z, double* ex, double* ey,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_spectra, dim3(1), dim3(DNT), 0, st, g, q, z, ex, ey);
}

}  // namespace fcns
