// FC spectral derivative along z without a context and without any device
// allocation: the transform's twiddle table and the continuation matrix are
// staged in a file-scope device array instead of context buffers.
//
// The array `scratch` holds, per call, [twiddles: tsize complex128][M: C*d
// float64].  Host code never passes its name to a kernel: on each device the
// address comes from hipGetSymbolAddress, taken once with that device current
// and kept per device.  Every call on a device shares that device's array, so
// calls that overlap on one device (several host threads, or several streams
// without ordering between them) race on the tables.
#include <mutex>

#include "../../include/fcns.h"
#include "kernels.hpp"

namespace fcns {

constexpr int NA_MAX_TW = 4096;   // complex128 twiddle entries
constexpr int NA_MAX_M = 256;     // float64 entries of M (C * d); passed by value
constexpr size_t NA_BYTES = NA_MAX_TW * sizeof(cpx<double>) + NA_MAX_M * sizeof(double);
constexpr int NA_MAX_DEV = 64;

static __device__ __align__(256) char scratch[NA_BYTES];

static std::mutex na_mutex;
static void* na_ptr[NA_MAX_DEV] = {};

// Device address of this device's scratch (looked up once per device).
static fcns_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NA_MAX_DEV) return FCNS_EDEVICE;
  std::lock_guard<std::mutex> lk(na_mutex);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FCNS_EDEVICE;
    na_ptr[dev] = p;
  }
  *out = na_ptr[dev];
  return FCNS_OK;
}

// The continuation matrix passed by value to the set-up kernel.
struct NAMatrix {
  double m[NA_MAX_M];
  int n;
};

// Twiddles of the Stockham plan (the same layout as the context's table: per
// stage with ns > 1 the factors exp(-2 pi i m k / (ns R)) as [m-1][k], per
// odd radix its R roots), and M, into the scratch.
__global__ void k_noalloc_tables(FFTPlan pl, NAMatrix mat, cpx<double>* tw, double* M) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  long long ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.r[s];
    if (pl.toff[s] >= 0) {
      const long long cnt = (long long)(R - 1) * ns, den = ns * R;
      for (long long e = tid; e < cnt; e += nt) {
        const long long m = 1 + e / ns, k = e % ns;
        const long long num = (m * k) % den;
        double sn, cs;
        sincospi(-2.0 * (double)num / (double)den, &sn, &cs);
        tw[pl.toff[s] + e] = mk(cs, sn);
      }
    }
    if (pl.coff[s] >= 0) {
      for (int q = tid; q < R; q += nt) {
        double sn, cs;
        sincospi(-2.0 * (double)q / (double)R, &sn, &cs);
        tw[pl.coff[s] + q] = mk(cs, sn);
      }
    }
    ns *= R;
  }
  if (pl.nst == 1 && pl.toff[0] < 0 && pl.coff[0] < 0 && tid == 0)
    tw[0] = mk(1.0, 0.0);   // a plan without factors keeps one unused entry
  for (int i = tid; i < mat.n; i += nt) M[i] = mat.m[i];
}

// Radices of the z transform (8s, 4s, 2s, then odd primes ascending; 288 as
// the compiled 16 x 18) and the table layout, without allocating.
static bool plan_for(int n, FFTPlan& pl, bool& big) {
  int rs[FFT_MAX_STAGES];
  int nr = 0, m = n;
  if (n == 288) {
    rs[nr++] = 16;
    rs[nr++] = 18;
    m = 1;
  }
  while (m % 8 == 0 && nr < FFT_MAX_STAGES) { rs[nr++] = 8; m /= 8; }
  while (m % 4 == 0 && nr < FFT_MAX_STAGES) { rs[nr++] = 4; m /= 4; }
  while (m % 2 == 0 && nr < FFT_MAX_STAGES) { rs[nr++] = 2; m /= 2; }
  for (int p = 3; m > 1 && p <= m; p += 2)
    while (m % p == 0 && nr < FFT_MAX_STAGES) {
      rs[nr++] = p;
      m /= p;
    }
  if (m != 1 || nr == 0) return false;
  pl = FFTPlan{};
  pl.n = n;
  pl.nst = nr;
  big = false;
  int size = 0;
  long long ns = 1;
  for (int s = 0; s < nr; ++s) {
    const int R = rs[s];
    pl.r[s] = R;
    if (R > 8) big = true;
    pl.toff[s] = -1;
    pl.coff[s] = -1;
    if (ns > 1) {
      pl.toff[s] = size;
      size += (int)((R - 1) * ns);
    }
    if (R % 2 == 1) {
      pl.coff[s] = size;
      size += R;
    }
    ns *= R;
  }
  pl.tsize = size > 0 ? size : 1;
  return true;
}

}  // namespace fcns

using namespace fcns;

extern "C" fcns_status fcns_fc_derivative_noalloc(int32_t nz, double lz, int32_t fc_d,
                                                  int32_t fc_C, const double* fc_table,
                                                  int32_t order, const double* in, int64_t nlines,
                                                  int64_t ps, int64_t ls, double* out,
                                                  void* hip_stream) {
  if (order != 1 && order != 2) return FCNS_EINVAL;
  if (fc_d < 2 || fc_C < 1 || nz < 2 * fc_d || !(lz > 0.0) || !fc_table) return FCNS_EINVAL;
  const int npr = nz + fc_C;
  if (npr % 2 || npr > z_max_npr()) return FCNS_EINVAL;   // N' even and <= 512
  if (fc_C * fc_d > NA_MAX_M) return FCNS_EINVAL;
  if (nlines < 0) return FCNS_EINVAL;
  if (nlines == 0) return FCNS_OK;
  if (!in || !out) return FCNS_EINVAL;
  FFTPlan pl;
  bool big = false;
  if (!plan_for(npr, pl, big) || pl.tsize > NA_MAX_TW) return FCNS_EINVAL;
  void* base = nullptr;
  fcns_status st = scratch_address(&base);
  if (st != FCNS_OK) return st;
  cpx<double>* tw = reinterpret_cast<cpx<double>*>(base);
  double* M = reinterpret_cast<double*>(reinterpret_cast<char*>(base) +
                                        NA_MAX_TW * sizeof(cpx<double>));
  // M_r = A_r Q_r^T in extended precision (App. B), as fcns_create forms it
  NAMatrix mat;
  mat.n = fc_C * fc_d;
  const double* Qr = fc_table;
  const double* Ar = fc_table + fc_d * fc_d;
  for (int i = 0; i < fc_C; ++i)
    for (int j = 0; j < fc_d; ++j) {
      long double acc = 0.0L;
      for (int k = 0; k < fc_d; ++k) acc += (long double)Ar[i * fc_d + k] * (long double)Qr[j * fc_d + k];
      mat.m[i * fc_d + j] = (double)acc;
    }
  hipStream_t stream = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_noalloc_tables, dim3(4), dim3(256), 0, stream, pl, mat, tw, M);
  if (hipGetLastError() != hipSuccess) return FCNS_EDEVICE;
  ZArgs a{};
  Geom& g = a.g;
  g.nz = nz;
  g.npr = npr;
  g.C = fc_C;
  g.d = fc_d;
  g.lz = lz;
  g.dz = lz / (nz - 1);
  g.lzp = npr * g.dz;
  g.kzs = 2.0 * M_PI / g.lzp;
  a.pl = pl;
  a.tw = tw;
  a.fc = M;
  a.nonfinite = nullptr;
  launch_fc_derivative(a, big, in, out, nlines, ps, ls, order, stream);
  return hipGetLastError() == hipSuccess ? FCNS_OK : FCNS_EDEVICE;
}
