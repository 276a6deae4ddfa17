// Wall-normal (z) kernels: FC-Gram continuation, FFTs of the continued
// lines, the RK stage combine with the splitting boundary conditions, and the
// pressure projection with its closed-form homogeneous part.
//
// Data layout (complex, x fastest): mixed (kx, ky, z) fields are
// [nz][ny][nkxp], continued spectral (kx, ky, kz) fields are [N'][ny][nkxp],
// with the kx row padded to nkxp (a multiple of 4, so that 4-line tiles of
// the y pass are 64-byte aligned).  A pencil is one (kx, ky) pair,
// p = ky * nkxp + kx; slots with kx >= nkx are padding and never touched.  A
// workgroup owns ZPB consecutive pencils and stages their lines in LDS as
// X[l * ZPB + pb] (pencil index fastest), so every global row access is ZPB
// consecutive complex values.
//
// Inverse transforms use IFFT(y) = conj(FFT(conj(y))) / N' with the
// conjugations folded into the surrounding loads and stores.
#include "kernels.hpp"

namespace fcns {

// ---------------------------------------------------------------- LDS layout
// [tw: plan table cpx<T>][M: C*d double, padded to 16 B][X0: NX cpx<T>][X1: NX cpx<T>]
// with NX = max(N' * ZPB, 4 * ZNT) (X1 also serves the reduction scratch).
template <typename T>
struct ZLds {
  cpx<T>* tw;
  double* M;
  cpx<T>* X0;
  cpx<T>* X1;
  __device__ ZLds(char* base, const Geom& g, int tsize) {
    tw = reinterpret_cast<cpx<T>*>(base);
    size_t off = ((tsize * sizeof(cpx<T>) + 15) / 16) * 16;
    M = reinterpret_cast<double*>(base + off);
    off += ((g.C * g.d * sizeof(double) + 15) / 16) * 16;
    X0 = reinterpret_cast<cpx<T>*>(base + off);
    const int nx = max(g.npr * ZPB, 4 * ZNT * (int)(sizeof(cpx<double>) / sizeof(cpx<T>)));
    X1 = X0 + nx;
  }
};

template <typename T>
size_t zshared_bytes(const Geom& g, int tsize) {
  const size_t a = (size_t)g.npr * ZPB, b = 4 * ZNT * (sizeof(cpx<double>) / sizeof(cpx<T>));
  const size_t nx = a > b ? a : b;
  return ((tsize * sizeof(cpx<T>) + 15) / 16) * 16 + ((g.C * g.d * sizeof(double) + 15) / 16) * 16 +
         2 * nx * sizeof(cpx<T>);
}

// Tables into LDS, in two halves so that a kernel can issue its own first
// loads in between: load() issues the global reads, store() writes LDS.  Up
// to 2 * ZNT entries each (the twiddle table always, as it has fewer than
// N' + 64 entries) the reads are all issued before any is waited for;
// larger continuation tables are copied by a loop inside store().
template <typename T>
struct ZTables {
  cpx<T> t0, t1;
  double m0, m1;
};

__device__ __forceinline__ bool ztab_fast(const ZArgs& a) {
  return a.pl.tsize <= 2 * ZNT && a.g.C * a.g.d <= 2 * ZNT;
}

template <typename T>
__device__ __forceinline__ ZTables<T> ztab_load(const ZArgs& a, int tid) {
  ZTables<T> t{};
  if (ztab_fast(a)) {
    const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
    const int nt = a.pl.tsize, nm = a.g.C * a.g.d;
    t.t0 = gtw[min(tid, nt - 1)];
    t.t1 = gtw[min(tid + ZNT, nt - 1)];
    t.m0 = a.fc[min(tid, nm - 1)];
    t.m1 = a.fc[min(tid + ZNT, nm - 1)];
  }
  return t;
}

template <typename T>
__device__ __forceinline__ void ztab_store(const ZTables<T> t, const ZLds<T>& s, const ZArgs& a,
                                           int tid) {
  const int nt = a.pl.tsize, nm = a.g.C * a.g.d;
  if (ztab_fast(a)) {
    if (tid < nt) s.tw[tid] = t.t0;
    if (tid + ZNT < nt) s.tw[tid + ZNT] = t.t1;
    if (tid < nm) s.M[tid] = t.m0;
    if (tid + ZNT < nm) s.M[tid + ZNT] = t.m1;
    return;
  }
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < nt; i += ZNT) s.tw[i] = gtw[i];
  for (int i = tid; i < nm; i += ZNT) s.M[i] = a.fc[i];
}

// The plain copy loop (measured faster than the split form for k_z_back).
template <typename T>
__device__ __forceinline__ void z_setup(const ZLds<T>& s, const ZArgs& a, int tid) {
  const cpx<T>* gtw = reinterpret_cast<const cpx<T>*>(a.tw);
  for (int i = tid; i < a.pl.tsize; i += ZNT) s.tw[i] = gtw[i];
  for (int i = tid; i < a.g.C * a.g.d; i += ZNT) s.M[i] = a.fc[i];
}

// Rows nz..nz+C-1 of every line: f^c = M_r f_r + M_l f_l with M_l = J M_r J
// (Sec. 3 continuation formula; App. B block form A f = A_l Q_l^T f_l +
// A_r Q_r^T f_r with M = A Q^T).
template <typename T>
__device__ __forceinline__ void z_extend_fma(cpx<T>* X, const double* __restrict__ M, int nz, int C,
                                             int d, int tid) {
  for (int e = tid; e < C * ZPB; e += ZNT) {
    const int i = e / ZPB, pb = e % ZPB;
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < d; ++j) {
      const double mr = M[i * d + j];
      const cpx<T> fr = X[(nz - d + j) * ZPB + pb];
      ar += mr * (double)fr.x;
      ai += mr * (double)fr.y;
    }
    for (int j = 0; j < d; ++j) {
      const double ml = M[(C - 1 - i) * d + (d - 1 - j)];
      const cpx<T> fl = X[j * ZPB + pb];
      ar += ml * (double)fl.x;
      ai += ml * (double)fl.y;
    }
    X[(nz + i) * ZPB + pb] = mk((T)ar, (T)ai);
  }
}

// The same continuation on the matrix cores: per workgroup the C x 2d matrix
// [M_r | M_l] times the 2d x 16 boundary values of its 8 pencils (real and
// imaginary parts as separate columns), as 2 row tiles x 3 k-steps of
// v_mfma_f64_16x16x4f64, one row tile per wavefront (C <= 32, d <= 6; rows and
// k-steps past C and 2d are zero).  Lane l supplies A[i][k] and B[k][j] with
// i, j = l % 16 and k = l / 16, and receives D[l / 16 + 4 r][l % 16],
// r = 0..3.  Accumulation is FP64 throughout.
typedef double zv4d __attribute__((ext_vector_type(4)));
static_assert(ZPB == 8, "the MFMA extension maps 8 pencils x (re, im) onto 16 columns");

__device__ __forceinline__ bool z_extend_mfma_ok(int C, int d) { return C <= 32 && d <= 6; }

__device__ __forceinline__ void z_extend_mfma(cpx<double>* X, const double* __restrict__ M, int nz,
                                              int C, int d, int tid) {
  // wavefront t (t = 0, 1) computes row tile t
  if (tid >= 128) return;
  const int t = tid >> 6, l = tid & 63, col = l % 16, kq = l / 16;
  const int pb = col >> 1, part = col & 1;
  const double* Xd = reinterpret_cast<const double*>(X);
  const int i = 16 * t + col;
  zv4d acc = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int k = 4 * s + kq;
    // B[k][col]: the right boundary rows nz-d..nz-1, then the left rows 0..d-1
    double b = 0.0, a = 0.0;
    if (k < d) b = Xd[2 * ((nz - d + k) * ZPB + pb) + part];
    else if (k < 2 * d) b = Xd[2 * ((k - d) * ZPB + pb) + part];
    if (i < C) {
      if (k < d) a = M[i * d + k];
      else if (k < 2 * d) a = M[(C - 1 - i) * d + (d - 1 - (k - d))];
    }
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  double* Xw = reinterpret_cast<double*>(X);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int io = 16 * t + kq + 4 * r;
    if (io < C) Xw[2 * ((nz + io) * ZPB + pb) + part] = acc[r];
  }
}

// FP64 lines take the matrix-core form where it applies.
template <typename T>
__device__ __forceinline__ void z_extend(cpx<T>* X, const double* __restrict__ M, int nz, int C,
                                         int d, int tid) {
  if constexpr (sizeof(T) == sizeof(double)) {
    if (z_extend_mfma_ok(C, d)) {
      z_extend_mfma(X, M, nz, C, d, tid);
      return;
    }
  }
  z_extend_fma<T>(X, M, nz, C, d, tid);
}

__device__ __forceinline__ void pencil_k(const Geom& g, long long p, double& kx_o, double& ky_o,
                                         double& kx_t, double& ky_t, int& ix, int& iy) {
  iy = (int)(p / g.nkxp);
  ix = (int)(p - (long long)iy * g.nkxp);
  kx_t = g.kxs * ix;
  kx_o = (2 * ix == g.nx) ? 0.0 : kx_t;
  ky_t = k_true(iy, g.ny, g.kys);
  ky_o = k_odd(iy, g.ny, g.kys);
}

// A pencil slot holds data when it is inside the array and not kx padding.
__device__ __forceinline__ bool pencil_valid(const Geom& g, long long p) {
  return p < g.npen && (int)(p % g.nkxp) < g.nkx;
}

// ---------------------------------------------------------------- z forward
// mixed -> continued spectral: F_z = FFT_N' o E (times the filter if asked).
template <typename T, class FP>
__global__ __launch_bounds__(ZNT) void k_z_fwd(ZArgs a, const cpx<double>* __restrict__ src,
                                               cpx<double>* __restrict__ dst, long long sfs,
                                               long long dfs, int filter) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const Geom& g = a.g;
  const ZLds<T> L(smem, g, a.pl.tsize);
  src += blockIdx.y * sfs;
  dst += blockIdx.y * dfs;
  const long long p0 = (long long)blockIdx.x * ZPB;
  z_setup<T>(L, a, tid);
  const int pb = tid % ZPB, lt = tid / ZPB;
  const long long p = p0 + pb;
  const bool pv = pencil_valid(g, p);
  for (int z = lt; z < g.nz; z += ZLS)
    L.X0[z * ZPB + pb] = pv ? cvt<T>(src[(long long)z * g.npen + p]) : zero<T>();
  __syncthreads();
  z_extend<T>(L.X0, L.M, g.nz, g.C, g.d, tid);
  __syncthreads();
  const cpx<T>* R = fft_run<T, ZPB, ZNT, false, FP>(L.X0, L.X1, ZPB, 1, a.pl, L.tw, tid);
  if (!pv) return;
  double sxy = 1.0;
  if (filter) {
    const int iy = (int)(p / g.nkxp), ix = (int)(p - (long long)iy * g.nkxp);
    sxy = a.sigy[iy] * a.sigx[ix];
  }
  for (int l = lt; l < g.npr; l += ZLS) {
    cpx<double> v = cvt<double>(R[l * ZPB + pb]);
    if (filter) v = v * (a.sigz[l] * sxy);
    dst[(long long)l * g.npen + p] = v;
  }
}

// ---------------------------------------------------------------- z back
// B_z = R o IFFT of one field whose continued rows this thread holds
// (keep[r] = row lt + r ZLS of pencil p0 + tid % ZPB, zero past N' and for
// padding pencils) into dst, and B_z(i k~z .) into dzdst when non-null.
// Every thread of the workgroup calls it; it ends with a barrier.
// NTS: streaming stores.
template <typename T, class FP, int OWN, bool NTS = false>
__device__ __forceinline__ void z_back_rows(const ZLds<T>& L, const ZArgs& a,
                                            const cpx<double> (&keep)[OWN], cpx<T>* dst,
                                            cpx<T>* dzdst, long long p0, int tid) {
  const Geom& g = a.g;
  const int npr = FP::dynamic ? g.npr : FP::n;
  const int tot = npr * ZPB;
  const int pb = tid % ZPB, lt = tid / ZPB;
  const long long p = p0 + pb;
  const bool pv = pencil_valid(g, p);
  const double inv = 1.0 / npr;
  const int npass = dzdst ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int e = tid + r * ZNT;
      if (e < tot) {
        cpx<double> v = keep[r];
        if (pass == 1) v = mul_i(v) * k_odd(lt + r * ZLS, npr, g.kzs);
        L.X0[e] = cvt<T>(conj(v));
      }
    }
    __syncthreads();
    const cpx<T>* R = fft_run<T, ZPB, ZNT, false, FP>(L.X0, L.X1, ZPB, 1, a.pl, L.tw, tid);
    cpx<T>* out = pass ? dzdst : dst;
    if (pv) {
      if constexpr (!FP::dynamic) {
        // compiled plans: LDS reads first (rows up to N' - 1 are in the
        // buffer), then the stores
        cpx<T> ov[OWN];
#pragma unroll
        for (int r = 0; r < OWN; ++r) ov[r] = R[min(lt + r * ZLS, npr - 1) * ZPB + pb];
#pragma unroll
        for (int r = 0; r < OWN; ++r)
          if (lt + r * ZLS < g.nz) {
            cpx<T>* o = out + (long long)(lt + r * ZLS) * g.npen + p;
            if constexpr (NTS)
              st_stream(o, conj(ov[r]) * (T)inv);
            else
              *o = conj(ov[r]) * (T)inv;
          }
      } else {
        for (int z = lt; z < g.nz; z += ZLS)
          out[(long long)z * g.npen + p] = conj(R[z * ZPB + pb]) * (T)inv;
      }
    }
    __syncthreads();
  }
}

// This thread's rows of one continued field (layout of z_back_rows); NT:
// the last read of them (streaming loads).
template <class FP, int OWN, bool NT = false>
__device__ __forceinline__ void load_rows(const ZArgs& a, const cpx<double>* src, long long p0,
                                          int tid, cpx<double> (&keep)[OWN]) {
  const Geom& g = a.g;
  const int npr = FP::dynamic ? g.npr : FP::n;
  const int pb = tid % ZPB, lt = tid / ZPB;
  const long long p = p0 + pb;
  const bool pv = pencil_valid(g, p);
#pragma unroll
  for (int r = 0; r < OWN; ++r) {
    const int l = lt + r * ZLS;
    if constexpr (NT)
      keep[r] = (pv && l < npr) ? ld_stream(src + (long long)l * g.npen + p) : zero<double>();
    else
      keep[r] = (pv && l < npr) ? src[(long long)l * g.npen + p] : zero<double>();
  }
}

// The step's non-finite check: every coefficient of the state passes here.
template <int OWN>
__device__ __forceinline__ void check_rows(const ZArgs& a, const cpx<double> (&keep)[OWN]) {
  if (!a.nonfinite) return;
  bool bad = false;
#pragma unroll
  for (int r = 0; r < OWN; ++r)
    bad = bad || !__builtin_isfinite(keep[r].x) || !__builtin_isfinite(keep[r].y);
  if (bad) *a.nonfinite = 1;
}

// continued spectral -> mixed: B_z = R o IFFT (and B_z(i k~z .) into dzdst).
template <typename T, class FP, int OWN>
__global__ __launch_bounds__(ZNT) void k_z_back(ZArgs a, const cpx<double>* __restrict__ src,
                                                cpx<T>* __restrict__ dst,
                                                cpx<T>* __restrict__ dzdst,
                                                long long sfs, long long mfs) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const ZLds<T> L(smem, a.g, a.pl.tsize);
  src += blockIdx.y * sfs;
  dst += blockIdx.y * mfs;
  if (dzdst) dzdst += blockIdx.y * mfs;
  const long long p0 = (long long)blockIdx.x * ZPB;
  z_setup<T>(L, a, tid);
  cpx<double> keep[OWN];
  load_rows<FP, OWN>(a, src, p0, tid, keep);
  check_rows<OWN>(a, keep);
  z_back_rows<T, FP, OWN>(L, a, keep, dst, dzdst, p0, tid);
}

// ---------------------------------------------------------------- stage A
// One field f (0..2 velocity, 3 temperature) of the pencil group at p0; T:
// transform type, TM: storage of the mixed-space inputs (NL, buoyancy).
// Sec. 4.4 steps 1-3 up to the FC-Gram transform of v*:
//   N = sigma F_z(NL);  S = V^t + c (N - diff |k|^2 W);  v* = B_z S, plus the
//   body force / buoyancy at the physical points, then the wall injection
//   v*_par = c grad_par p_prev (theta = 0) and V* = F_z v*.
// TABLES: also stage the plan and continuation tables in LDS (the first
// field a workgroup handles).  SPECBUOY: s.buoy[f] is the other field's
// continued state W (theta for w, w for theta) and the buoyancy enters S as
// c gamma W_other, which B_z maps onto c gamma times its physical values (the
// term of Sec. 7 added at the physical points); otherwise s.buoy[f] holds
// the other field's mixed values, added after the inverse transform.
// Ends with this thread's stores; the caller places a barrier before the
// LDS is used again.
// KEEPOUT: the result rows are also left in keep (the row layout of
// z_back_rows, zero past N' and for padding pencils); STORE = false: they
// are only left there.
template <typename T, typename TM, class FP, int OWN, bool WV, bool SPECBUOY,
          bool KEEPOUT = false, bool STORE = true>
// nl_in: this field's nonlinear-term rows, already loaded (else they are
// loaded here); nl_out: receives field fnext's rows, loaded before the last
// transform so that they arrive while it runs; cs_out likewise receives the
// rows of the continued field cs_next (rows past N' clamped; the layout of
// z_back_rows).
__device__ __forceinline__ void z_stageA_field(const ZLds<T>& L, const ZArgs& a,
                                               const StageAArgs& s, int f, long long p0, int tid,
                                               bool tables, cpx<double>* keep = nullptr,
                                               const cpx<TM>* nl_in = nullptr, int fnext = -1,
                                               cpx<TM>* nl_out = nullptr,
                                               const cpx<double>* cs_next = nullptr,
                                               cpx<double>* cs_out = nullptr) {
  // a fresh copy of the thread index: the row offsets derived from it are
  // recomputed per field rather than kept live from one field to the next
  asm volatile("" : "+v"(tid));
  const Geom& g = a.g;
  const int npr = FP::dynamic ? g.npr : FP::n;
  ZTables<T> tab{};
  if (tables) tab = ztab_load<T>(a, tid);
  const cpx<TM>* nl = reinterpret_cast<const cpx<TM>*>(s.nl[f]);
  const cpx<double>* vt = s.vt[f];
  const cpx<double>* w = s.w[f];
  const cpx<TM>* buoy = SPECBUOY ? nullptr : reinterpret_cast<const cpx<TM>*>(s.buoy[f]);
  const cpx<double>* wbuoy = SPECBUOY ? reinterpret_cast<const cpx<double>*>(s.buoy[f]) : nullptr;
  const double c = s.c;
  const double diff = (f == 3) ? s.kappa : s.nu;
  const double inv = 1.0 / npr;
  const int pb = tid % ZPB, lt = tid / ZPB;
  const long long p = p0 + pb;
  const bool pv = pencil_valid(g, p);
  double kxo, kyo, kxt, kyt;
  int ix, iy;
  pencil_k(g, pv ? p : 0, kxo, kyo, kxt, kyt, ix, iy);
  const double kh2 = kxt * kxt + kyt * kyt;
  cpx<T>* R = L.X0;
  // All of this thread's loads before the first transform are issued before
  // any is waited for: the nonlinear term's rows (rows past nz and invalid
  // pencils read an in-bounds slot that is then discarded), then the
  // continued state and filter factors, in flight during the transform.
  // (the fused pass streams them: they are read once, V* is read back)
  constexpr bool NT = SPECBUOY;
  auto ld = [](const auto* q) {
    if constexpr (NT)
      return ld_stream(q);
    else
      return *q;
  };
  cpx<TM> nr[OWN];
  const long long pc = pv ? p : 0;
  if (nl_in) {
#pragma unroll
    for (int r = 0; r < OWN; ++r) nr[r] = nl_in[r];
  } else {
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int z = min(lt + r * ZLS, g.nz - 1);
      nr[r] = ld(nl + (long long)z * g.npen + pc);
    }
  }
  // keep these loads ahead of the ones below (loads complete in order, so a
  // later one issued first would hold up the LDS writes of these rows)
  __builtin_amdgcn_sched_barrier(0);
  // (WV: W is V^t itself, as at the first RK stage; it is not loaded twice)
  cpx<double> vtr[OWN], wr[OWN];
  double sgr[OWN];
#pragma unroll
  for (int r = 0; r < OWN; ++r) {
    const int l = min(lt + r * ZLS, npr - 1);  // rows past N' are never used
    const long long gi = (long long)l * g.npen + pc;
    vtr[r] = ld(vt + gi);
    if constexpr (!WV) wr[r] = ld(w + gi);
    sgr[r] = a.sigz[l];
  }
  // (rows z >= nz store zero to a continuation row, rewritten by the
  // extension after the barrier, so that no load is tied to a branch)
  if (tables) ztab_store<T>(tab, L, a, tid);
#pragma unroll
  for (int r = 0; r < OWN; ++r) {
    const int z = lt + r * ZLS;
    L.X0[min(z, npr - 1) * ZPB + pb] = (pv && z < g.nz) ? cvt<T>(nr[r]) : zero<T>();
  }
  const double sxy = a.sigy[iy] * a.sigx[ix];
  // 1. nonlinear term at the physical points (loaded above), continued,
  // transformed
  __syncthreads();
  z_extend<T>(L.X0, L.M, g.nz, g.C, g.d, tid);
  __syncthreads();
  R = fft_run<T, ZPB, ZNT, false, FP>(L.X0, L.X1, ZPB, 1, a.pl, L.tw, tid);
  // 2. S = V^t + c (sigma N - diff |k|^2 W) [+ c gamma W_other], conjugated
  // for the inverse (the other field's rows are loaded now, and added after
  // the combine has released the registers of the state rows)
  const double cg = c * s.gamma;
  cpx<double> bsr[SPECBUOY ? OWN : 1];
  if constexpr (SPECBUOY) {
    if (wbuoy) {
#pragma unroll
      for (int r = 0; r < OWN; ++r)
        bsr[r] = ld(wbuoy + (long long)min(lt + r * ZLS, npr - 1) * g.npen + pc);
    }
  }
#pragma unroll
  for (int r = 0; r < OWN; ++r) {
    const int l = lt + r * ZLS;
    if (l < npr) {
      const int e = l * ZPB + pb;
      cpx<double> S = zero<double>();
      if (pv) {
        const double kzt = k_true(l, npr, g.kzs);
        const double k2 = kh2 + kzt * kzt;
        const double sig = sgr[r] * sxy;
        S = vtr[r] + (cvt<double>(R[e]) * sig - (WV ? vtr[r] : wr[r]) * (diff * k2)) * c;
      }
      if constexpr (SPECBUOY) {
        if (wbuoy && pv) S = S + bsr[r] * cg;
      }
      L.X0[e] = cvt<T>(conj(S));
    }
  }
  // the buoyancy rows and wall values of this thread, in flight during the
  // inverse transform
  cpx<double> br[OWN];
  if (buoy) {
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int z = lt + r * ZLS;
      br[r] = (pv && z < g.nz) ? cvt<double>(buoy[(long long)z * g.npen + p]) : zero<double>();
    }
  }
  const bool has_w0 = lt == 0, has_w1 = (g.nz - 1) % ZLS == lt;
  cpx<double> gw0 = zero<double>(), gw1 = zero<double>();
  if (pv && f < 2) {
    if (has_w0) gw0 = s.gwall[(0 * 2 + f) * g.npen + p];
    if (has_w1) gw1 = s.gwall[(1 * 2 + f) * g.npen + p];
  }
  __syncthreads();
  R = fft_run<T, ZPB, ZNT, false, FP>(L.X0, L.X1, ZPB, 1, a.pl, L.tw, tid);
  // 3. v* at the physical points: forcing, buoyancy, wall injection;
  // continued and transformed
#pragma unroll
  for (int r = 0; r < OWN; ++r) {
    const int z = lt + r * ZLS;
    if (z < g.nz) {
      const int e = z * ZPB + pb;
      cpx<double> v = zero<double>();
      if (pv) {
        v = conj(cvt<double>(R[e])) * inv;
        if (f == 0 && p == 0) v.x += c * s.forcing_sum;
        if (buoy) v = v + br[r] * cg;
        if (z == 0 || z == g.nz - 1) {
          if (f < 2) v = ((z == 0) ? gw0 : gw1) * c;
          if (f == 3) v = zero<double>();
        }
      }
      L.X0[e] = cvt<T>(v);
    }
  }
  __syncthreads();
  z_extend<T>(L.X0, L.M, g.nz, g.C, g.d, tid);
  if (nl_out) {
    const cpx<TM>* nln = reinterpret_cast<const cpx<TM>*>(s.nl[fnext]);
#pragma unroll
    for (int r = 0; r < OWN; ++r)
      nl_out[r] = ld(nln + (long long)min(lt + r * ZLS, g.nz - 1) * g.npen + pc);
  }
  if (cs_out) {
#pragma unroll
    for (int r = 0; r < OWN; ++r)
      cs_out[r] = cs_next[(long long)min(lt + r * ZLS, npr - 1) * g.npen + pc];
  }
  __syncthreads();
  R = fft_run<T, ZPB, ZNT, false, FP>(L.X0, L.X1, ZPB, 1, a.pl, L.tw, tid);
  // compiled plans: all of this thread's LDS reads first, then the stores
  // (the rolled loop waits for each read in turn; it measured faster on the
  // small run-time-plan grids)
  cpx<double>* out = s.out[f];
  if constexpr (KEEPOUT) {
#pragma unroll
    for (int r = 0; r < OWN; ++r) {
      const int l = lt + r * ZLS;
      keep[r] = (pv && l < npr) ? cvt<double>(R[l * ZPB + pb]) : zero<double>();
    }
    if (STORE && pv) {
#pragma unroll
      for (int r = 0; r < OWN; ++r)
        if (lt + r * ZLS < npr) {
          // (not read again by the workgroup)
          cpx<double>* o = out + (long long)(lt + r * ZLS) * g.npen + p;
          if constexpr (NT)
            st_stream(o, keep[r]);
          else
            *o = keep[r];
        }
    }
    return;
  }
  if (pv) {
    if constexpr (!FP::dynamic) {
      cpx<double> ov[OWN];
#pragma unroll
      for (int r = 0; r < OWN; ++r) ov[r] = cvt<double>(R[min(lt + r * ZLS, npr - 1) * ZPB + pb]);
#pragma unroll
      for (int r = 0; r < OWN; ++r)
        if (lt + r * ZLS < npr) out[(long long)(lt + r * ZLS) * g.npen + p] = ov[r];
    } else {
      for (int l = lt; l < npr; l += ZLS) out[(long long)l * g.npen + p] = cvt<double>(R[l * ZPB + pb]);
    }
  }
}

// One field per blockIdx.y.
template <typename T, typename TM, class FP, int OWN, bool WV>
__global__ __launch_bounds__(ZNT) void k_z_stageA(ZArgs a, StageAArgs s) {
  extern __shared__ __align__(16) char smem[];
  const ZLds<T> L(smem, a.g, a.pl.tsize);
  z_stageA_field<T, TM, FP, OWN, WV, false>(L, a, s, blockIdx.y, (long long)blockIdx.x * ZPB,
                                            threadIdx.x, true);
}

// ---------------------------------------------------------------- stage B
// Pressure projection of V* (Sec. 4.2; Sec. 4.4 steps 3-5) in increment units
// phi = c p:
//   s = (k~ . V*) / |k~|^2, grad phi^I = k~ s (phi^I = -i s);
//   b, t = wall values of B_z(V*_z - k~z s);
//   gamma = |k~_h|, A = (t - b E)/(gamma (1 - E^2)), B = -(b - t E)/(...),
//   E = exp(-gamma Lz); H = grad(A e^{gamma (z - Lz)} + B e^{-gamma z})
//   (gamma = 0: H = (0, 0, D), D = (b + t)/2);
//   V = V* - k~ s - F_z H; next-stage wall gradient (k~ B_z s + H)_par / c.
// The two exponentials are continued as the real and imaginary parts of one
// line; F_z(e+ + i e-) splits into F_z e+ and F_z e- by conjugate symmetry.
// HOLD > 0 (N' <= HOLD * ZLS): V* is read once and held in registers (HOLD
// rows per thread); HOLD = 0: V* is streamed twice (wall sums, then the
// update).  KEEP (needs HOLD): the projected rows are also left in vk, in
// the row layout of z_back_rows, for the back transform of the result in
// the same workgroup; otherwise the mixed v, dv/dz of the result come from
// k_z_back.  TABLES: stage the plan and continuation tables in LDS.
// coef (ZPB * 5 entries) and gam_s (ZPB) are LDS scratch.
// KF >= 0 (needs HOLD): V* of field KF is not read but taken from kv, this
// thread's rows in the layout of z_back_rows, and kv receives the field's
// projected rows in their place.
// KP >= 0 (needs HOLD): V* of field KP is taken from kp (rows already
// loaded) instead of being read here.
template <typename T, class FP, int HOLD, bool KEEP, int KF = -1, int KP = -1>
__device__ __forceinline__ void z_stageB_body(const ZLds<T>& L, const ZArgs& a,
                                              const StageBArgs& s, long long p0, int tid,
                                              cpx<double>* coef, double* gam_s, bool tables,
                                              cpx<double> (&vk)[3][KEEP ? HOLD : 1],
                                              cpx<double>* kv = nullptr,
                                              const cpx<double>* kp = nullptr) {
  static_assert(!KEEP || HOLD > 0, "KEEP needs the rows held in registers");
  static_assert(KF < 0 || HOLD > 0, "KF needs the rows held in registers");
  const Geom& g = a.g;
  const int npr = FP::dynamic ? g.npr : FP::n;
  const int pb_me = tid % ZPB, lt = tid / ZPB;
  const long long p_me = p0 + pb_me;
  const bool valid_me = pencil_valid(g, p_me);
  ZTables<T> tab{};
  if (tables) tab = ztab_load<T>(a, tid);
  const cpx<double>* gtw = a.tw64;
  const double inv = 1.0 / npr;
  const bool pm = s.pmix != nullptr;
  // rows of this thread: l = lt + r ZLS, r < nr
  constexpr int HR = HOLD > 0 ? HOLD : 1;
  const int nr = HOLD > 0 ? HOLD : (npr - lt + ZLS - 1) / ZLS;

  double kxo, kyo, kxt, kyt;
  int ix, iy;
  pencil_k(g, valid_me ? p_me : 0, kxo, kyo, kxt, kyt, ix, iy);
  const double kh2 = kxo * kxo + kyo * kyo;

  // 1. wall sums of B_z(V*_z - k~z s) and B_z(s)
  cpx<double> sb = zero<double>(), st = zero<double>(), s0 = zero<double>(),
              s1 = zero<double>();
  // root index l (nz - 1) mod N', stepped with l
  const int step = (int)(((long long)ZLS * (g.nz - 1)) % npr);
  const int ei0 = (int)(((long long)lt * (g.nz - 1)) % npr);
  // HOLD > 0: the roots of this thread's rows and V* itself, all loads issued
  // together (rows of an invalid pencil, and rows past N', read an in-bounds
  // slot and are never used)
  cpx<double> hv[3][HR], etr[HR];
  if constexpr (HOLD > 0) {
#pragma unroll
    for (int r = 0, ei = ei0; r < HOLD; ++r, ei = (ei + step >= npr) ? ei + step - npr : ei + step)
      etr[r] = conj(gtw[ei]);
#pragma unroll
    for (int r = 0; r < HOLD; ++r) {
      const long long gi =
          valid_me ? (long long)min(lt + r * ZLS, npr - 1) * g.npen + p_me : 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) hv[i][r] = (i == KF) ? kv[r] : (i == KP) ? kp[r] : s.vs[i][gi];
    }
  }
  if (tables) ztab_store<T>(tab, L, a, tid);
  if (valid_me) {
    int ei = ei0;
#pragma unroll(HR)
    for (int r = 0; r < nr; ++r, ei = (ei + step >= npr) ? ei + step - npr : ei + step) {
      const int l = lt + r * ZLS;
      if (l >= npr) continue;
      cpx<double> V0, V1, V2;
      if constexpr (HOLD > 0) {
        V0 = hv[0][r];
        V1 = hv[1][r];
        V2 = hv[2][r];
      } else {
        const long long gi = (long long)l * g.npen + p_me;
        V0 = s.vs[0][gi];
        V1 = s.vs[1][gi];
        V2 = s.vs[2][gi];
      }
      const double kz = k_odd(l, npr, g.kzs);
      const double k2 = kh2 + kz * kz;
      cpx<double> sv = zero<double>();
      if (k2 > 0.0) sv = (V0 * kxo + V1 * kyo + V2 * kz) * (1.0 / k2);
      const cpx<double> rz = V2 - sv * kz;
      // e^{+2 pi i l (nz-1)/N'} = conj(root[l (nz-1) mod N'])
      cpx<double> et;
      if constexpr (HOLD > 0)
        et = etr[r];
      else
        et = conj(gtw[ei]);
      sb = sb + rz;
      st = st + rz * et;
      s0 = s0 + sv;
      s1 = s1 + sv * et;
    }
  }
  cpx<double>* red = reinterpret_cast<cpx<double>*>(L.X1);
  red[tid * 4 + 0] = sb;
  red[tid * 4 + 1] = st;
  red[tid * 4 + 2] = s0;
  red[tid * 4 + 3] = s1;
  __syncthreads();
  if (tid < ZPB * 4) {
    const int pb = tid % ZPB, q = tid / ZPB;
    cpx<double> acc = zero<double>();
    for (int m = 0; m < ZNT / ZPB; ++m) acc = acc + red[(pb + m * ZPB) * 4 + q];
    coef[pb * 5 + q] = acc * inv;  // b, t, s0, s1
  }
  __syncthreads();
  // 2. homogeneous coefficients and the wall gradient for the next stage
  if (tid < ZPB) {
    const int pb = tid;
    const long long p = p0 + pb;
    double qkxo, qkyo, qkxt, qkyt;
    int qix, qiy;
    const bool qv = pencil_valid(g, p);
    pencil_k(g, qv ? p : 0, qkxo, qkyo, qkxt, qkyt, qix, qiy);
    const cpx<double> b = coef[pb * 5 + 0], t = coef[pb * 5 + 1];
    const cpx<double> sw0 = coef[pb * 5 + 2], sw1 = coef[pb * 5 + 3];
    const double gam = sqrt(qkxo * qkxo + qkyo * qkyo);
    cpx<double> A = zero<double>(), B = zero<double>(), D = zero<double>();
    double E = 0.0;
    if (gam > 0.0) {
      E = exp(-gam * g.lz);
      const double den = 1.0 / (gam * (1.0 - E * E));
      A = (t - b * E) * den;
      B = (b - t * E) * (-den);
    } else {
      D = (b + t) * 0.5;
    }
    gam_s[pb] = gam;
    if (qv && s.gwall) {
      // H_par at the walls: i k~ (A e+ + B e-) with e+(0) = E, e-(0) = 1,
      // e+(Lz) = 1, e-(Lz) = E
      const cpx<double> h0 = mul_i(A * E + B), h1 = mul_i(A + B * E);
      const double ic = 1.0 / s.c;
      s.gwall[(0 * 2 + 0) * g.npen + p] = (sw0 + h0) * (qkxo * ic);
      s.gwall[(0 * 2 + 1) * g.npen + p] = (sw0 + h0) * (qkyo * ic);
      s.gwall[(1 * 2 + 0) * g.npen + p] = (sw1 + h1) * (qkxo * ic);
      s.gwall[(1 * 2 + 1) * g.npen + p] = (sw1 + h1) * (qkyo * ic);
    }
    coef[pb * 5 + 0] = A;
    coef[pb * 5 + 1] = B;
    coef[pb * 5 + 2] = D;
  }
  __syncthreads();
  const cpx<double> A = coef[pb_me * 5 + 0], B = coef[pb_me * 5 + 1], D = coef[pb_me * 5 + 2];
  const double gam = gam_s[pb_me];

  // 3. F_z(e+ + i e-) (gamma = 0: F_z(1))
  for (int z = lt; z < g.nz; z += ZLS) {
    const double zz = z * g.dz;
    L.X0[z * ZPB + pb_me] =
        (gam > 0.0) ? mk((T)exp(gam * (zz - g.lz)), (T)exp(-gam * zz)) : mk((T)1, (T)0);
  }
  __syncthreads();
  z_extend<T>(L.X0, L.M, g.nz, g.C, g.d, tid);
  __syncthreads();
  const cpx<T>* R = fft_run<T, ZPB, ZNT, false, FP>(L.X0, L.X1, ZPB, 1, a.pl, L.tw, tid);
  cpx<T>* Xo = (R == L.X0) ? L.X1 : L.X0;
  // 4. V = V* - k~ s - H^ (V* held or streamed again), store the continued state
  if constexpr (KEEP) {
#pragma unroll
    for (int r = 0; r < HOLD; ++r)
#pragma unroll
      for (int i = 0; i < 3; ++i) vk[i][r] = zero<double>();
  }
#pragma unroll(HR)
  for (int r = 0; r < nr; ++r) {
    const int l = lt + r * ZLS;
    if (l >= npr) continue;
    const int e = l * ZPB + pb_me;
    if (!valid_me) {
      if (pm) Xo[e] = zero<T>();
      continue;
    }
    const long long gi = (long long)l * g.npen + p_me;
    cpx<double> V0, V1, V2;
    if constexpr (HOLD > 0) {
      V0 = hv[0][r];
      V1 = hv[1][r];
      V2 = hv[2][r];
    } else {
      V0 = s.vs[0][gi];
      V1 = s.vs[1][gi];
      V2 = s.vs[2][gi];
    }
    const int lm = (l == 0) ? 0 : npr - l;
    const cpx<double> xl = cvt<double>(R[e]), xm = conj(cvt<double>(R[lm * ZPB + pb_me]));
    const cpx<double> ep = (xl + xm) * 0.5;
    const cpx<double> em = mul_mi(xl - xm) * 0.5;
    const double kz = k_odd(l, npr, g.kzs);
    const double k2 = kh2 + kz * kz;
    cpx<double> sv = zero<double>();
    if (k2 > 0.0) sv = (V0 * kxo + V1 * kyo + V2 * kz) * (1.0 / k2);
    cpx<double> hx = zero<double>(), hy = zero<double>(), hz;
    if (gam > 0.0) {
      const cpx<double> sym = A * ep + B * em;
      hx = mul_i(sym) * kxo;
      hy = mul_i(sym) * kyo;
      hz = (A * ep - B * em) * gam;
    } else {
      hz = D * ep;
    }
    const cpx<double> n0 = V0 - sv * kxo - hx, n1 = V1 - sv * kyo - hy, n2 = V2 - sv * kz - hz;
    // (field KF's rows go back in kv and are not read again: streaming store)
    if constexpr (KF == 0) st_stream(&s.vout[0][gi], n0); else s.vout[0][gi] = n0;
    if constexpr (KF == 1) st_stream(&s.vout[1][gi], n1); else s.vout[1][gi] = n1;
    if constexpr (KF == 2) st_stream(&s.vout[2][gi], n2); else s.vout[2][gi] = n2;
    if constexpr (KF >= 0) kv[r] = (KF == 0) ? n0 : (KF == 1) ? n1 : n2;
    if constexpr (KEEP) {
      vk[0][r] = n0;
      vk[1][r] = n1;
      vk[2][r] = n2;
    }
    if (pm) Xo[e] = cvt<T>(conj(mul_mi(sv)));  // phi^I = -i s, conjugated
  }
  if (pm) {
    // 5. pressure in mixed space: (B_z(-i s) + phi^H) / c
    __syncthreads();
    const cpx<T>* P =
        fft_run<T, ZPB, ZNT, false, FP>(Xo, (Xo == L.X0) ? L.X1 : L.X0, ZPB, 1, a.pl, L.tw, tid);
    if (valid_me)
      for (int z = lt; z < g.nz; z += ZLS) {
        const double zz = z * g.dz;
        cpx<double> ph;
        if (gam > 0.0)
          ph = A * exp(gam * (zz - g.lz)) + B * exp(-gam * zz);
        else
          ph = D * zz;
        s.pmix[(long long)z * g.npen + p_me] =
            (conj(cvt<double>(P[z * ZPB + pb_me])) * inv + ph) * (1.0 / s.c);
      }
  }
}

template <typename T, class FP, int HOLD>
__global__ __launch_bounds__(ZNT) void k_z_stageB(ZArgs a, StageBArgs s) {
  extern __shared__ __align__(16) char smem[];
  __shared__ cpx<double> coef[ZPB * 5];  // b, t, s0, s1 then A, B, D
  __shared__ double gam_s[ZPB];
  const ZLds<T> L(smem, a.g, a.pl.tsize);
  cpx<double> vk[3][1];
  z_stageB_body<T, FP, HOLD, false>(L, a, s, (long long)blockIdx.x * ZPB, threadIdx.x, coef,
                                    gam_s, true, vk);
}

// ---------------------------------------------------------------- one fused z pass
// The whole z pass of one RK stage for a group of ZPB pencils (FP64): stage
// A for every transported field (velocity into s.out[0..2] as V*, except
// the last one, which stays in registers; theta as its new state; the
// buoyancy in spectral form), the projection of V* in place (stage B, V*
// read back while it is still in the caches), and the back transforms of
// the new state (v, dv/dz of every field into the mixed arrays; theta's and
// the last velocity field's from the rows still in registers).  The
// outputs must not alias the inputs of another field (true when the stage
// writes the other state buffer, as both stages of o = 2 do); W of the
// other field feeds the buoyancy.  Each pencil group is independent, so V*
// never has to reach HBM: it is written, read back and overwritten by the
// same workgroup.
// The fused z pass of one pencil group at p0 (every thread of the workgroup).
template <class FP, int OWN, bool WV>
__device__ __forceinline__ void z_pass_group(const ZLds<double>& L, const ZArgs& a,
                                             const StageAArgs& sa, const StageBArgs& sb,
                                             const ZBackArgs& zb, int nf, long long p0, int tid,
                                             cpx<double>* coef, double* gam_s) {
  // one field after the other (the field index a constant in each copy);
  // theta first: its new state is final after stage A, so its back
  // transforms follow at once from the rows still in registers
  // (each field's nonlinear-term rows are loaded during the previous field's
  // last transform)
  cpx<double> pre_w[OWN], pre_u[OWN], pre_v[OWN];
  if (nf == 4) {
    cpx<double> keep[OWN];
    z_stageA_field<double, double, FP, OWN, WV, true, true>(L, a, sa, 3, p0, tid, true, keep,
                                                            nullptr, 2, pre_w);
    __syncthreads();
    check_rows<OWN>(a, keep);
    z_back_rows<double, FP, OWN, true>(L, a, keep, zb.mv + 6 * zb.ms, zb.mv + 7 * zb.ms, p0,
                                       tid);
  }
  // then w (its buoyancy reads theta's W again, soon after theta did), u,
  // and v, whose V* goes to the projection in registers without a store
  if (nf != 4) {   // (no theta to load them during)
    const int pb = tid % ZPB, lt = tid / ZPB;
    const long long pc = pencil_valid(a.g, p0 + pb) ? p0 + pb : 0;
    const cpx<double>* nlw = reinterpret_cast<const cpx<double>*>(sa.nl[2]);
#pragma unroll
    for (int r = 0; r < OWN; ++r)
      pre_w[r] = ld_stream(nlw + (long long)min(lt + r * ZLS, a.g.nz - 1) * a.g.npen + pc);
  }
  z_stageA_field<double, double, FP, OWN, WV, true>(L, a, sa, 2, p0, tid, nf != 4, nullptr,
                                                    pre_w, 0, pre_u);
  __syncthreads();
  z_stageA_field<double, double, FP, OWN, WV, true>(L, a, sa, 0, p0, tid, false, nullptr, pre_u,
                                                    1, pre_v);
  __syncthreads();
  // (w's V* rows for the projection are loaded during v's last transform)
  cpx<double> vstar1[OWN], vstar2[OWN];
  z_stageA_field<double, double, FP, OWN, WV, true, true, false>(L, a, sa, 1, p0, tid, false,
                                                                  vstar1, pre_v, -1, nullptr,
                                                                  sa.out[2], vstar2);
  __syncthreads();
  cpx<double> vk[3][1];
  z_stageB_body<double, FP, OWN, false, 1, 2>(L, a, sb, p0, tid, coef, gam_s, false, vk, vstar1,
                                              vstar2);
  __syncthreads();
  // v's new state is in registers; each thread reads back the rows of u and
  // w it has just written (cache hits)
  check_rows<OWN>(a, vstar1);
  z_back_rows<double, FP, OWN, true>(L, a, vstar1, zb.mv + 2 * zb.ms, zb.mv + 3 * zb.ms, p0,
                                     tid);
  for (int f = 0; f < 3; f += 2) {
    cpx<double> keep[OWN];
    load_rows<FP, OWN, true>(a, sa.out[f], p0, tid, keep);
    check_rows<OWN>(a, keep);
    z_back_rows<double, FP, OWN, true>(L, a, keep, zb.mv + (2 * f) * zb.ms,
                                       zb.mv + (2 * f + 1) * zb.ms, p0, tid);
  }
}

template <class FP, int OWN, bool WV>
__global__ __launch_bounds__(ZNT, 2) void k_z_pass(ZArgs a, StageAArgs sa, StageBArgs sb,
                                                   ZBackArgs zb, int nf) {
  extern __shared__ __align__(16) char smem[];
  __shared__ cpx<double> coef[ZPB * 5];
  __shared__ double gam_s[ZPB];
  const ZLds<double> L(smem, a.g, a.pl.tsize);
  z_pass_group<FP, OWN, WV>(L, a, sa, sb, zb, nf, (long long)blockIdx.x * ZPB, threadIdx.x,
                            coef, gam_s);
}

// The fused z pass of several problems of different shapes in one launch:
// workgroup b serves problem r with d[r].wg0 <= b < d[r + 1].wg0, pencil
// group b - d[r].wg0 of it, with that problem's own geometry, plan, tables
// and buffers.  Each workgroup runs exactly the code of k_z_pass (FP and OWN
// cover every problem of the batch; rows past a problem's N' are masked).
template <class FP, int OWN>
__global__ __launch_bounds__(ZNT, 2) void k_z_pass_batch(const ZPassDesc* d, int n) {
  extern __shared__ __align__(16) char smem[];
  __shared__ cpx<double> coef[ZPB * 5];
  __shared__ double gam_s[ZPB];
  int r = 0;
  while (r + 1 < n && (long long)blockIdx.x >= d[r + 1].wg0) ++r;
  const ZPassDesc& D = d[r];
  const ZLds<double> L(smem, D.a.g, D.a.pl.tsize);
  z_pass_group<FP, OWN, false>(L, D.a, D.sa, D.sb, D.zb, D.nf,
                               ((long long)blockIdx.x - D.wg0) * ZPB, threadIdx.x, coef, gam_s);
}

// ---------------------------------------------------------------- fc_extend
// Strided real lines, one thread per line.
__global__ __launch_bounds__(256) void k_fc_extend(const double* __restrict__ in, long long nlines,
                                                   long long ips, long long ils,
                                                   double* __restrict__ out, long long ops,
                                                   long long ols, int nz, int C, int d,
                                                   const double* __restrict__ M) {
  const long long line = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= nlines) return;
  const double* f = in + line * ils;
  double* o = out + line * ols;
  for (int s = 0; s < nz; ++s) o[s * ops] = f[s * ips];
  for (int i = 0; i < C; ++i) {
    double acc = 0.0;
    for (int j = 0; j < d; ++j) acc += M[i * d + j] * f[(nz - d + j) * ips];
    for (int j = 0; j < d; ++j) acc += M[(C - 1 - i) * d + (d - 1 - j)] * f[j * ips];
    o[(nz + i) * ops] = acc;
  }
}

// ---------------------------------------------------------------- fc_derivative
// Two real lines per complex line (line 2q real part, 2q+1 imaginary part):
// the multipliers i k~z (Nyquist zeroed) and -kz^2 map real lines to real
// lines, so the packed transform differentiates both at once.
template <class FP>
__global__ __launch_bounds__(ZNT) void k_fc_derivative(ZArgs a, const double* __restrict__ in,
                                                       double* __restrict__ out, long long nlines,
                                                       long long ps, long long ls, int order) {
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const Geom& g = a.g;
  const ZLds<double> L(smem, g, a.pl.tsize);
  z_setup<double>(L, a, tid);
  const long long q0 = (long long)blockIdx.x * ZPB;
  for (int e = tid; e < g.nz * ZPB; e += ZNT) {
    const int z = e / ZPB, pb = e % ZPB;
    const long long l0 = 2 * (q0 + pb), l1 = l0 + 1;
    const double re = (l0 < nlines) ? in[l0 * ls + z * ps] : 0.0;
    const double im = (l1 < nlines) ? in[l1 * ls + z * ps] : 0.0;
    L.X0[e] = mk(re, im);
  }
  __syncthreads();
  z_extend<double>(L.X0, L.M, g.nz, g.C, g.d, tid);
  __syncthreads();
  const cpx<double>* R = L.X0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int e = tid; e < g.npr * ZPB; e += ZNT) {
        const int l = e / ZPB;
        cpx<double> v = R[e];
        if (order == 1) {
          v = mul_i(v) * k_odd(l, g.npr, g.kzs);
        } else {
          const double k = k_true(l, g.npr, g.kzs);
          v = v * (-k * k);
        }
        L.X0[e] = conj(v);
      }
      __syncthreads();
    }
    R = fft_run<double, ZPB, ZNT, false, FP>(L.X0, L.X1, ZPB, 1, a.pl, L.tw, tid);
  }
  const double inv = 1.0 / g.npr;
  for (int e = tid; e < g.nz * ZPB; e += ZNT) {
    const int z = e / ZPB, pb = e % ZPB;
    const long long l0 = 2 * (q0 + pb), l1 = l0 + 1;
    const cpx<double> v = conj(R[e]) * inv;
    if (l0 < nlines) out[l0 * ls + z * ps] = v.x;
    if (l1 < nlines) out[l1 * ls + z * ps] = v.y;
  }
}

// ---------------------------------------------------------------- launchers
static int pick_own(int npr) {
  const int need = (npr * ZPB + ZNT - 1) / ZNT;
  if (need <= 4) return 4;
  if (need <= 9) return 9;
  return 16;
}

int z_max_npr() { return 16 * ZNT / ZPB; }

#define FCNS_OWN_SWITCH(OWNV, CALL)                 \
  switch (OWNV) {                                   \
    case 4: { constexpr int OWN = 4; CALL; } break; \
    case 9: { constexpr int OWN = 9; CALL; } break; \
    default: { constexpr int OWN = 16; CALL; } break; \
  }

// Compile-time plan for N' = 288 (nz = 257 with C = 31); other lengths run
// the run-time engine.
using P288 = SPlan<16, 18>;
static bool z_static_288(const ZArgs& a) { return a.g.npr == 288 && plan_is(a.pl, {16, 18}); }
// N' = 282 (nz = 257 with C = 25) in the radix order 47, 2, 3 (the prime
// stage first, so it needs no twiddle pass): compiled as well
using P282 = SPlan<47, 2, 3>;
static bool z_static_282(const ZArgs& a) { return a.g.npr == 282 && plan_is(a.pl, {47, 2, 3}); }

void launch_z_fwd(const ZArgs& a, bool big, const cpx<double>* src, cpx<double>* dst,
                  long long sfs, long long dfs, int nfields, int filter, hipStream_t st) {
  dim3 grid((unsigned)((a.g.npen + ZPB - 1) / ZPB), nfields);
  const size_t sh = zshared_bytes<double>(a.g, a.pl.tsize);
  if (z_static_288(a))
    FCNS_LAUNCH((k_z_fwd<double, P288>), grid, dim3(ZNT), sh, st, a, src, dst, sfs, dfs, filter);
  else if (z_static_282(a))
    FCNS_LAUNCH((k_z_fwd<double, P282>), grid, dim3(ZNT), sh, st, a, src, dst, sfs, dfs, filter);
  else if (big)
    FCNS_LAUNCH((k_z_fwd<double, DynPlan<true>>), grid, dim3(ZNT), sh, st, a, src, dst, sfs, dfs,
                filter);
  else
    FCNS_LAUNCH((k_z_fwd<double, DynPlan<false>>), grid, dim3(ZNT), sh, st, a, src, dst, sfs, dfs,
                filter);
}


template <typename T>
void launch_z_back(const ZArgs& a, bool big, const cpx<double>* src, cpx<T>* dst, cpx<T>* dzdst,
                   long long sfs, long long mfs, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((a.g.npen + ZPB - 1) / ZPB), nfields);
  const size_t sh = zshared_bytes<T>(a.g, a.pl.tsize);
  const int own = pick_own(a.g.npr);
  if (z_static_288(a)) {
    FCNS_LAUNCH((k_z_back<T, P288, 9>), grid, dim3(ZNT), sh, st, a, src, dst, dzdst, sfs, mfs);
  } else if (z_static_282(a)) {
    FCNS_LAUNCH((k_z_back<T, P282, 9>), grid, dim3(ZNT), sh, st, a, src, dst, dzdst, sfs, mfs);
  } else if (big) {
    FCNS_OWN_SWITCH(own, FCNS_LAUNCH((k_z_back<T, DynPlan<true>, OWN>), grid, dim3(ZNT), sh, st,
                                     a, src, dst, dzdst, sfs, mfs))
  } else {
    FCNS_OWN_SWITCH(own, FCNS_LAUNCH((k_z_back<T, DynPlan<false>, OWN>), grid, dim3(ZNT), sh, st,
                                     a, src, dst, dzdst, sfs, mfs))
  }
}
template void launch_z_back<double>(const ZArgs&, bool, const cpx<double>*, cpx<double>*,
                                    cpx<double>*, long long, long long, int, hipStream_t);
template void launch_z_back<float>(const ZArgs&, bool, const cpx<double>*, cpx<float>*,
                                   cpx<float>*, long long, long long, int, hipStream_t);

template <typename TM>
void launch_z_stageA(const ZArgs& a, bool big, const StageAArgs& s, int nfields, hipStream_t st) {
  using T = double;
  dim3 grid((unsigned)((a.g.npen + ZPB - 1) / ZPB), nfields);
  const size_t sh = zshared_bytes<T>(a.g, a.pl.tsize);
  const int own = pick_own(a.g.npr);
  if (z_static_288(a)) {
    bool wv = true;  // W is V^t for every field (the first RK stage)
    for (int f = 0; f < nfields; ++f) wv = wv && s.w[f] == s.vt[f];
    if (wv)
      FCNS_LAUNCH((k_z_stageA<T, TM, P288, 9, true>), grid, dim3(ZNT), sh, st, a, s);
    else
      FCNS_LAUNCH((k_z_stageA<T, TM, P288, 9, false>), grid, dim3(ZNT), sh, st, a, s);
  } else if (z_static_282(a)) {
    FCNS_LAUNCH((k_z_stageA<T, TM, P282, 9, false>), grid, dim3(ZNT), sh, st, a, s);
  } else if (big) {
    FCNS_OWN_SWITCH(own, FCNS_LAUNCH((k_z_stageA<T, TM, DynPlan<true>, OWN, false>), grid, dim3(ZNT),
                                     sh, st, a, s))
  } else {
    FCNS_OWN_SWITCH(own, FCNS_LAUNCH((k_z_stageA<T, TM, DynPlan<false>, OWN, false>), grid,
                                     dim3(ZNT), sh, st, a, s))
  }
}
template void launch_z_stageA<double>(const ZArgs&, bool, const StageAArgs&, int, hipStream_t);
template void launch_z_stageA<float>(const ZArgs&, bool, const StageAArgs&, int, hipStream_t);

void launch_z_stageB(const ZArgs& a, bool big, const StageBArgs& s, hipStream_t st) {
  dim3 grid((unsigned)((a.g.npen + ZPB - 1) / ZPB), 1);
  const size_t sh = zshared_bytes<double>(a.g, a.pl.tsize);
  const int own = pick_own(a.g.npr);
  if (z_static_288(a))
    FCNS_LAUNCH((k_z_stageB<double, P288, 288 / ZLS>), grid, dim3(ZNT), sh, st, a, s);
  else if (z_static_282(a))
    FCNS_LAUNCH((k_z_stageB<double, P282, 9>), grid, dim3(ZNT), sh, st, a, s);
  // run-time plans: V* held in registers (9 rows per thread) for
  // 128 < N' <= 288 without primes above 7 (224: 0.145 -> 0.113 ms at side
  // 192; with such primes it would leave one wave per SIMD, and 4 rows for
  // N' <= 128 measured no faster than streaming V* twice)
  else if (big)
    FCNS_LAUNCH((k_z_stageB<double, DynPlan<true>, 0>), grid, dim3(ZNT), sh, st, a, s);
  else if (own == 9)
    FCNS_LAUNCH((k_z_stageB<double, DynPlan<false>, 9>), grid, dim3(ZNT), sh, st, a, s);
  else
    FCNS_LAUNCH((k_z_stageB<double, DynPlan<false>, 0>), grid, dim3(ZNT), sh, st, a, s);
}

bool z_pass_fits(const ZArgs& a) { return pick_own(a.g.npr) <= 9; }

size_t z_pass_lds(const ZArgs& a) { return zshared_bytes<double>(a.g, a.pl.tsize); }
long long z_pass_groups(const ZArgs& a) { return (a.g.npen + ZPB - 1) / ZPB; }

void launch_z_pass_batch(const ZPassDesc* d, int n, long long groups, int max_npr, bool big,
                         size_t lds, hipStream_t st) {
  dim3 grid((unsigned)groups);
  if (pick_own(max_npr) <= 4) {
    if (big)
      FCNS_LAUNCH((k_z_pass_batch<DynPlan<true>, 4>), grid, dim3(ZNT), lds, st, d, n);
    else
      FCNS_LAUNCH((k_z_pass_batch<DynPlan<false>, 4>), grid, dim3(ZNT), lds, st, d, n);
  } else {
    if (big)
      FCNS_LAUNCH((k_z_pass_batch<DynPlan<true>, 9>), grid, dim3(ZNT), lds, st, d, n);
    else
      FCNS_LAUNCH((k_z_pass_batch<DynPlan<false>, 9>), grid, dim3(ZNT), lds, st, d, n);
  }
}

void launch_z_pass(const ZArgs& a, bool big, const StageAArgs& sa, const StageBArgs& sb,
                   const ZBackArgs& zb, int nfields, hipStream_t st) {
  dim3 grid((unsigned)((a.g.npen + ZPB - 1) / ZPB));
  const size_t sh = zshared_bytes<double>(a.g, a.pl.tsize);
  const int own = pick_own(a.g.npr);
  if (z_static_288(a)) {
    bool wv = true;  // W is V^t for every field (the first RK stage)
    for (int f = 0; f < nfields; ++f) wv = wv && sa.w[f] == sa.vt[f];
    if (wv)
      FCNS_LAUNCH((k_z_pass<P288, 9, true>), grid, dim3(ZNT), sh, st, a, sa, sb, zb, nfields);
    else
      FCNS_LAUNCH((k_z_pass<P288, 9, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb, nfields);
  } else if (z_static_282(a)) {
    FCNS_LAUNCH((k_z_pass<P282, 9, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb, nfields);
  } else if (own == 9 && plan_is(a.pl, {8, 4, 7})) {
    // N' = 224, 160, 128, 96 and 64 (the sides 192, 128, 96, 64 and 32 with
    // C = 31): compiled plans, N' / 32 rows per thread
    FCNS_LAUNCH((k_z_pass<SPlan<8, 4, 7>, 7, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                nfields);
  } else if (own == 9 && plan_is(a.pl, {8, 4, 5})) {
    FCNS_LAUNCH((k_z_pass<SPlan<8, 4, 5>, 5, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                nfields);
  } else if (own == 4 && plan_is(a.pl, {8, 8, 2})) {
    FCNS_LAUNCH((k_z_pass<SPlan<8, 8, 2>, 4, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                nfields);
  } else if (own == 4 && plan_is(a.pl, {8, 4, 3})) {
    FCNS_LAUNCH((k_z_pass<SPlan<8, 4, 3>, 3, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                nfields);
  } else if (own == 4 && plan_is(a.pl, {8, 8})) {
    FCNS_LAUNCH((k_z_pass<SPlan<8, 8>, 2, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                nfields);
  } else if (big) {
    if (own <= 4)
      FCNS_LAUNCH((k_z_pass<DynPlan<true>, 4, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                  nfields);
    else
      FCNS_LAUNCH((k_z_pass<DynPlan<true>, 9, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                  nfields);
  } else {
    if (own <= 4)
      FCNS_LAUNCH((k_z_pass<DynPlan<false>, 4, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                  nfields);
    else
      FCNS_LAUNCH((k_z_pass<DynPlan<false>, 9, false>), grid, dim3(ZNT), sh, st, a, sa, sb, zb,
                  nfields);
  }
}

void launch_fc_extend(const double* in, long long nlines, long long ips, long long ils, double* out,
                      long long ops, long long ols, int nz, int C, int d, const double* M,
                      hipStream_t st) {
  const int nt = 256;
  dim3 grid((unsigned)((nlines + nt - 1) / nt));
  FCNS_LAUNCH(k_fc_extend, grid, dim3(nt), 0, st, in, nlines, ips, ils, out, ops, ols, nz,
                     C, d, M);
}

void launch_fc_derivative(const ZArgs& a, bool big, const double* in, double* out,
                          long long nlines, long long ps, long long ls, int order,
                          hipStream_t st) {
  const long long nq = (nlines + 1) / 2;
  dim3 grid((unsigned)((nq + ZPB - 1) / ZPB));
  const size_t sh = zshared_bytes<double>(a.g, a.pl.tsize);
  if (z_static_288(a))
    FCNS_LAUNCH(k_fc_derivative<P288>, grid, dim3(ZNT), sh, st, a, in, out, nlines, ps, ls, order);
  else if (big)
    FCNS_LAUNCH(k_fc_derivative<DynPlan<true>>, grid, dim3(ZNT), sh, st, a, in, out, nlines, ps, ls,
                order);
  else
    FCNS_LAUNCH(k_fc_derivative<DynPlan<false>>, grid, dim3(ZNT), sh, st, a, in, out, nlines, ps, ls,
                order);
}



}  // namespace fcns
