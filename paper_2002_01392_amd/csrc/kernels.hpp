// Internal launch interface between the C-ABI host code and the HIP kernels.
#pragma once
#include "fcns_common.hpp"
#include "fft_lds.hpp"

#include <initializer_list>

namespace fcns {

// z kernels: ZPB pencils per workgroup of ZNT threads
constexpr int ZPB = 8;
constexpr int ZNT = 256;
constexpr int ZLS = ZNT / ZPB;  // rows a thread steps over (its pencil is tid % ZPB)
// y kernels: YL lines (consecutive kx) per workgroup
constexpr int YL = 4;
constexpr int YNT = 256;
constexpr long long Y_GRID = 1024;  // persistent y workgroups per field
// x kernels: XR rows per workgroup (XR/2 complex lines); nx <= XNT
constexpr int XR = 8;
constexpr int XNT = 512;

// Does the run-time plan have exactly these radices (in this order)?
inline bool plan_is(const FFTPlan& pl, std::initializer_list<int> rs) {
  if (pl.nst != (int)rs.size()) return false;
  int s = 0;
  for (int r : rs)
    if (pl.r[s++] != r) return false;
  return true;
}

struct ZArgs {
  Geom g;
  FFTPlan pl;             // N'-point plan (lines = ZPB, threads = ZNT)
  const void* tw;         // N' twiddles in the transform precision
  const cpx<double>* tw64;  // N' twiddles in FP64 (wall sums)
  const double* fc;       // M_r, C x d row-major
  const double* sigx;     // filter factors per direction (nkx, ny, N')
  const double* sigy;
  const double* sigz;
  int* nonfinite;         // non-null: set to 1 by k_z_back when the state it
                          // reads holds a NaN or an infinity
};

// Mixed-space arrays (nl, buoy) hold cpx<T> of the kernel's transform type T.
struct StageAArgs {
  const void* nl[4];          // mixed nonlinear term per field
  const cpx<double>* vt[4];   // continued state at t
  const cpx<double>* w[4];    // continued state of the previous stage
  cpx<double>* out[4];        // V* (velocity) or Theta^(j) (temperature)
  const void* buoy[4];        // mixed theta (for w) / w (for theta), or null
  const cpx<double>* gwall;   // [2 walls][2 comps][npen], p units
  double c;                   // stage coefficient c_j
  double nu, kappa, gamma;
  double forcing_sum;         // body force times nx*ny (mixed (0,0) mode)
};

struct StageBArgs {
  const cpx<double>* vs[3];   // V*
  cpx<double>* vout[3];       // projected continued velocity
  cpx<double>* gwall;         // out: next-stage wall tangential gradient (or null)
  cpx<double>* pmix;          // out: mixed pressure (or null)
  double c;
};

struct YArgs {
  int ny, nkx, nkxp;
  double kys;
  FFTPlan pl;        // ny-point plan (lines = YL, threads = YNT)
  const void* tw;    // ny twiddles
  long long grid;    // persistent workgroups per field (0: Y_GRID)
  int noprefetch;    // 1: load each tile when needed instead of one tile ahead
  int blk;           // bit 0: src, bit 1: dst in the blocked (kx, ky) layout
  int lines;         // lines per tile: YL, or 8 where y_wide_tiles (whole 128-byte rows)
};
// 8-line tiles (512 threads) exist for the compiled 512-point plan
bool y_wide_tiles(const YArgs& a);

struct XArgs {
  int nx, nkx, nkxp, ny;
  double kxs;
  FFTPlan pl;        // nx-point plan (lines = XR/2, threads = XNT)
  const void* tw;    // nx twiddles
  int variant;       // x pass with products: 0 default, 1 tiled 4 rows x 256, 2 tiled 8 x 512,
                     // 3 tiled 8 rows x nx threads (nx <= 256)
  int blk_in;        // 1: x pass with products reads xyb in the blocked (kx, y) layout
                     // (variant 0 at nx = 512 and 256 only)
};

int z_max_npr();
size_t y_lds_bytes(int ny, int tsize, size_t elem, int lines = YL);  // LDS of one y workgroup
size_t z_lds_bytes(const Geom& g);

// Dynamic LDS above 64 KiB needs an explicit per-kernel opt-in.
#define FCNS_LAUNCH(K, GRID, BLOCK, SH, ST, ...)        \
  do {                                                  \
    allow_lds(K, SH);                                   \
    hipLaunchKernelGGL(K, GRID, BLOCK, SH, ST, __VA_ARGS__); \
  } while (0)
template <typename K>
inline void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_z_fwd(const ZArgs& a, bool big, const cpx<double>* src, cpx<double>* dst,
                  long long sfs, long long dfs, int nfields, int filter, hipStream_t st);
// T: transform type and mixed-space storage (double, or float for the mixed
// precision step); the continued state is always double.  The ZArgs / YArgs /
// XArgs twiddle table must be the one of type T.
template <typename T>
void launch_z_back(const ZArgs& a, bool big, const cpx<double>* src, cpx<T>* dst, cpx<T>* dzdst,
                   long long sfstride, long long mfstride, int nfields, hipStream_t st);
// stage A transforms in FP64 always (it forms V*, which the projection
// needs to full precision); TM is the storage of its mixed-space inputs.
template <typename TM>
void launch_z_stageA(const ZArgs& a, bool big, const StageAArgs& s, int nfields, hipStream_t st);
void launch_z_stageB(const ZArgs& a, bool big, const StageBArgs& s, hipStream_t st);

// The fused z pass of one FP64 stage (stage A for every field, the
// projection, the back transforms of the new state): sa.out velocity slots
// receive V* and then the projected state (sb.vs = sb.vout = sa.out),
// sa.buoy[2] / [3] are the continued W of theta / w, zb.mv gets v_f, dv_f/dz
// at slots 2f, 2f + 1.  z_pass_fits: N' small enough for the rows a thread
// keeps in registers (N' <= 288).
struct ZBackArgs {
  cpx<double>* mv;   // mixed v_f at slot 2f, dv_f/dz at 2f + 1
  long long ms;      // mixed field stride (elements)
};
bool z_pass_fits(const ZArgs& a);
void launch_z_pass(const ZArgs& a, bool big, const StageAArgs& sa, const StageBArgs& sb,
                   const ZBackArgs& zb, int nfields, hipStream_t st);

// One launch of the fused z pass over several problems (device array of n
// descriptors; wg0 = first workgroup of each problem, ascending from 0;
// groups = total workgroups).  Every problem runs the run-time plan engine
// (big: some plan has a prime radix above 7); max_npr picks the rows per
// thread; lds = the largest z_pass_lds of the batch.
struct ZPassDesc {
  ZArgs a;
  StageAArgs sa;
  StageBArgs sb;
  ZBackArgs zb;
  int nf;
  long long wg0;
};
size_t z_pass_lds(const ZArgs& a);
long long z_pass_groups(const ZArgs& a);
void launch_z_pass_batch(const ZPassDesc* d, int n, long long groups, int max_npr, bool big,
                         size_t lds, hipStream_t st);
void launch_fc_extend(const double* in, long long nlines, long long ips, long long ils, double* out,
                      long long ops, long long ols, int nz, int C, int d, const double* M,
                      hipStream_t st);
void launch_fc_derivative(const ZArgs& a, bool big, const double* in, double* out,
                          long long nlines, long long ps, long long ls, int order,
                          hipStream_t st);

// y: lines are (plane, kx) pairs, element ky; arrays [nplanes][ny][nkxp].
// mode 0: dst = FFT (inverse scaled by 1/ny); mode 1 (inverse only): also
// dst2 = inverse FFT of i k~y times the input.
template <typename T>
void launch_y(const YArgs& a, bool big, bool inv, int mode, const cpx<T>* src, cpx<T>* dst,
              cpx<T>* dst2, long long sfstride, long long dfstride, int nplanes, int nfields,
              hipStream_t st);
// x: rows are (plane, y) pairs; physical rows of nx reals <-> nkx complex
// (row stride nkxp).
void launch_x_r2c(const XArgs& a, bool big, const double* phys, cpx<double>* xy,
                  long long pfstride, long long xfstride, long long nrows, int nfields,
                  hipStream_t st);
void launch_x_c2r(const XArgs& a, bool big, const cpx<double>* xy, double* phys,
                  long long xfstride, long long pfstride, long long nrows, int nfields,
                  hipStream_t st);
// fused c2r + products + r2c: xyb holds, per field f, q_f, dq_f/dy, dq_f/dz at
// field slots 3f, 3f+1, 3f+2; nl gets -(v.grad) q_f at slot f.
template <typename T>
void launch_x_nl(const XArgs& a, bool big, const cpx<T>* xyb, cpx<T>* nl, long long fstride,
                 long long nrows, int nfields, hipStream_t st);
// the x pass with products can read xyb in the blocked layout (a.blk_in)
bool x_reads_blocked(const XArgs& a);

// diagnostics (mv: slots 2f = q_f, 2f+1 = dq_f/dz, stride ms)
void launch_diag_planes(const Geom& g, const cpx<double>* mv, long long ms, int nf, double* out,
                        hipStream_t st);
void launch_spectra(const Geom& g, const cpx<double>* q, int z, double* ex, double* ey,
                    hipStream_t st);

// small helpers
void launch_fill(cpx<double>* p, long long n, hipStream_t st);
void launch_sub_mean00(cpx<double>* pmix, long long npen, int nz, double scale, hipStream_t st);

}  // namespace fcns
