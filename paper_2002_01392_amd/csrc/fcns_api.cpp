// Host side of the C ABI: problem validation, FFT plans, tables, buffers and
// the sequence of kernel launches for each entry point.
#include <math.h>

#include <cmath>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/fcns.h"
#include "kernels.hpp"

using namespace fcns;

struct fcns_ctx {
  fcns_problem prob;
  hipStream_t stream = nullptr;
  Geom g{};
  int nf = 3;          // transported fields
  bool big_z = false, big_x = false, big_y = false;
  FFTPlan plz{}, plx{}, ply{};
  // device tables
  cpx<double>* twz = nullptr;   // plan twiddle tables
  cpx<double>* twx = nullptr;
  cpx<double>* twy = nullptr;
  cpx<double>* rootz = nullptr; // N' roots of unity (wall sums)
  bool mixed = false;           // FP32 transforms and mixed-space arrays in rk_step
  cpx<float>* twz_f = nullptr;  // the plan tables rounded to FP32 (mixed precision)
  cpx<float>* twx_f = nullptr;
  cpx<float>* twy_f = nullptr;
  double* fcM = nullptr;
  double* sigx = nullptr;
  double* sigy = nullptr;
  double* sigz = nullptr;
  std::vector<double> hostM;
  // device buffers (complex, counts in elements)
  long long S = 0, M = 0;  // one continued spectral / one mixed field
  cpx<double>* P = nullptr;    // V^t (nf fields)
  cpx<double>* Q = nullptr;    // V^(j) (nf fields)
  cpx<double>* VS = nullptr;   // V* / scratch (nf fields)
  cpx<double>* MV = nullptr;   // mixed v_f, dv_f/dz at slots 2f, 2f+1 (cpx<float> when mixed)
  cpx<double>* MVT = nullptr;  // scratch copy of MV for the standalone calls
  cpx<double>* XYB = nullptr;  // (kx, y, z): q_f, dq_f/dy, dq_f/dz at 3f..3f+2 (rk_step: T)
  cpx<double>* NLB = nullptr;  // nonlinear term (nf fields; rk_step: T)
  cpx<double>* PM = nullptr;   // mixed pressure
  cpx<double>* GW = nullptr;   // wall tangential gradient [2][2][npen]
  cpx<double>* GWT = nullptr;  // scratch wall gradient
  double* DG = nullptr;        // diagnostics: per-plane sums [nz][5], then spectra
  // non-finite check of the state: a flag in pinned, host-coherent memory,
  // raised by the z back transform of every stage (dflag: its device
  // address), read by the host once the work is done; no copy per step
  int* dflag = nullptr;
  int* hflag = nullptr;
  int check_mode = FCNS_CHECK_SYNC;
  // one RK step captured as a HIP graph (fcns_rk_graph), for one dt
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  double graph_dt = 0.0;
  // autotuned launch choices (fcns_autotune)
  int xvar = 0;
  long long ygrid = 0;   // y launches of one transform per tile
  int ynopf = 0;
  long long ygrid1 = 0;  // y back with d/dy (two transforms per tile)
  int ynopf1 = 0;
  int ylines = 4;        // lines (kx columns) per y tile: 4, or 8 (whole 128-byte rows)
  int ylines1 = 4;
  bool xyblk = false;    // rk_step's (kx, y) intermediates in the blocked layout (y back
                         // transforms write 4-column blocks contiguously; the x pass reads them)
  int slab = 0;          // > 0: the y / x passes of rk_step run slab by slab, this
                         // many z planes at a time (0: whole arrays)
  bool zfuse = false;    // FP64 stages writing the other state buffer: one fused z
                         // pass (chosen by fcns_autotune where it is faster)
  bool has_state = false;
  bool has_pressure = false;
  std::string err;
  // kernel timing (HIP events around the rk_step launches of the classes in
  // tmask, bit i = class i)
  bool timing = false;
  uint32_t tmask = 0;
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  Rec cur{};
  double tms[16] = {};
  long long tcnt[16] = {};
};

// Kernel classes timed by fcns_set_timing.
enum { T_YBACK_DY = 0, T_YBACK_DZ, T_XNL, T_YFWD, T_ZSTAGEA, T_ZSTAGEB, T_ZBACK, T_ZPASS,
       T_XYSLAB, T_NCLS };
static const char* kTimingNames[T_NCLS] = {"y_back_dy", "y_back_dz", "x_nl", "y_fwd",
                                           "z_stageA", "z_stageB", "z_back", "z_pass",
                                           "xy_slabs"};

static void timing_flush(fcns_ctx* c) {
  if (c->recs.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (const auto& r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->tms[r.cls] += ms;
      c->tcnt[r.cls] += 1;
    }
  }
  c->recs.clear();
  c->evnext = 0;
}

static void tbeg(fcns_ctx* c, int cls) {
  c->cur.cls = -1;
  if (!c->timing || !((c->tmask >> cls) & 1u)) return;
  if (c->evnext + 2 > c->evpool.size()) timing_flush(c);
  c->cur.cls = cls;
  c->cur.a = c->evpool[c->evnext++];
  (void)hipEventRecord(c->cur.a, c->stream);
}

static void tend(fcns_ctx* c) {
  if (!c->timing || c->cur.cls < 0) return;
  c->cur.b = c->evpool[c->evnext++];
  (void)hipEventRecord(c->cur.b, c->stream);
  c->recs.push_back(c->cur);
}

static std::string g_create_err;

static fcns_status fail(fcns_ctx* c, fcns_status st, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_create_err = msg;
  return st;
}

static fcns_status check_hip(fcns_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return FCNS_OK;
  return fail(c, FCNS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static fcns_status check_launch(fcns_ctx* c, const char* what) {
  return check_hip(c, hipGetLastError(), what);
}

// ---------------------------------------------------------------- plans
// Radices 8 first, then 4, 2 and odd primes ascending (at most 12 stages).
// Also lays out the twiddle table: per stage with ns > 1 the factors
// w^{m k} = exp(-2 pi i m k / (ns R)) as [m-1][k], and per odd-radix stage its
// R roots exp(-2 pi i q / R).
static std::vector<int> default_radices(int n) {
  int m = n;
  std::vector<int> rs;
  while (m % 8 == 0) { rs.push_back(8); m /= 8; }
  while (m % 4 == 0) { rs.push_back(4); m /= 4; }
  while (m % 2 == 0) { rs.push_back(2); m /= 2; }
  for (int p = 3; m > 1 && p <= m; p += 2)
    while (m % p == 0) {
      rs.push_back(p);
      m /= p;
    }
  if (m != 1) rs.clear();
  return rs;
}

static bool make_plan_order(int n, const std::vector<int>& rs, FFTPlan& pl, bool& big,
                            std::vector<cpx<double>>& table) {
  memset(&pl, 0, sizeof(pl));
  pl.n = n;
  big = false;
  long long prod = 1;
  for (int r : rs) prod *= r;
  if (rs.empty() || prod != n || (int)rs.size() > FFT_MAX_STAGES) return false;
  pl.nst = (int)rs.size();
  const long double pi = 3.141592653589793238462643383279502884L;
  auto root = [&](long long num, long long den) {
    const long double a = -2.0L * pi * (long double)num / (long double)den;
    return mk((double)cosl(a), (double)sinl(a));
  };
  table.clear();
  long long ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = rs[s];
    pl.r[s] = R;
    if (R > 8) big = true;  // 29, 47 and other primes
    pl.toff[s] = -1;
    pl.coff[s] = -1;
    if (ns > 1) {
      pl.toff[s] = (int)table.size();
      for (int mm = 1; mm < R; ++mm)
        for (long long k = 0; k < ns; ++k) table.push_back(root((long long)mm * k, ns * R));
    }
    if (R % 2 == 1) {
      pl.coff[s] = (int)table.size();
      for (int q = 0; q < R; ++q) table.push_back(root(q, R));
    }
    ns *= R;
  }
  if (table.empty()) table.push_back(mk(1.0, 0.0));
  pl.tsize = (int)table.size();
  return true;
}

static bool make_plan(int n, FFTPlan& pl, bool& big, std::vector<cpx<double>>& table) {
  return make_plan_order(n, default_radices(n), pl, big, table);
}

// The z plan: 288 (nz = 257 with C = 31) runs the compiled 16 x 18 transform
// (two register codelets, two LDS passes); radices 16 and 18 exist only
// there, never in a run-time plan.
static std::vector<int> z_radices(int n) {
  if (n == 288) return {16, 18};
  return default_radices(n);
}

static std::vector<cpx<double>> roots(int n) {
  std::vector<cpx<double>> t(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int q = 0; q < n; ++q) {
    const long double a = -2.0L * pi * (long double)q / (long double)n;
    t[q] = mk((double)cosl(a), (double)sinl(a));
  }
  return t;
}

static std::vector<double> filter_table(int n, int nstore, bool half, double beta, double two_p) {
  std::vector<double> s(nstore);
  for (int i = 0; i < nstore; ++i) {
    const int m = half ? i : ((2 * i < n) ? i : i - n);
    const double eta = 2.0 * fabs((double)m) / (double)n;
    s[i] = exp(-beta * pow(eta, two_p));
  }
  return s;
}

template <typename T>
static fcns_status upload(fcns_ctx* c, T** dst, const T* src, size_t n) {
  if (hipMalloc((void**)dst, n * sizeof(T)) != hipSuccess)
    return fail(c, FCNS_ENOMEM, "device allocation of a table failed");
  return check_hip(c, hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice), "table upload");
}

static fcns_status alloc(fcns_ctx* c, cpx<double>** p, long long n) {
  if (hipMalloc((void**)p, (size_t)n * sizeof(cpx<double>)) != hipSuccess)
    return fail(c, FCNS_ENOMEM, "device allocation failed");
  return FCNS_OK;
}

static void free_all(fcns_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
  c->evpool.clear();
  void* ps[] = {c->twz, c->twx, c->twy, c->twz_f, c->twx_f, c->twy_f, c->rootz, c->fcM, c->sigx, c->sigy, c->sigz, c->P, c->Q,
                c->VS, c->MV, c->MVT, c->XYB, c->NLB, c->PM, c->GW, c->GWT, c->DG};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (c->hflag) (void)hipHostFree(c->hflag);
}

// f32: the twiddle table of the FP32 kernels
static ZArgs zargs(const fcns_ctx* c, bool f32 = false) {
  ZArgs a;
  memset(&a, 0, sizeof(a));  // padding too: batch descriptors are compared bytewise
  a.g = c->g;
  a.pl = c->plz;
  a.tw = f32 ? (const void*)c->twz_f : (const void*)c->twz;
  a.tw64 = c->rootz;
  a.fc = c->fcM;
  a.sigx = c->sigx;
  a.sigy = c->sigy;
  a.sigz = c->sigz;
  a.nonfinite = nullptr;
  return a;
}
static YArgs yargs(const fcns_ctx* c, bool f32 = false, bool dy = false) {
  YArgs a{};
  a.ny = c->g.ny;
  a.nkx = c->g.nkx;
  a.nkxp = c->g.nkxp;
  a.kys = c->g.kys;
  a.pl = c->ply;
  a.tw = f32 ? (const void*)c->twy_f : (const void*)c->twy;
  a.grid = dy ? c->ygrid1 : c->ygrid;
  a.noprefetch = dy ? c->ynopf1 : c->ynopf;
  a.lines = dy ? c->ylines1 : c->ylines;
  return a;
}
static XArgs xargs(const fcns_ctx* c, bool f32 = false) {
  XArgs a{};
  a.nx = c->g.nx;
  a.nkx = c->g.nkx;
  a.nkxp = c->g.nkxp;
  a.ny = c->g.ny;
  a.kxs = c->g.kxs;
  a.pl = c->plx;
  a.tw = f32 ? (const void*)c->twx_f : (const void*)c->twx;
  a.variant = c->xvar;
  return a;
}

// ---------------------------------------------------------------- create
extern "C" fcns_status fcns_create(const fcns_problem* prob, void* hip_stream, fcns_ctx** out) {
  if (!out) return fail(nullptr, FCNS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!prob) return fail(nullptr, FCNS_EINVAL, "problem is NULL");
  const fcns_problem& p = *prob;
  if (p.nx < 4 || p.ny < 4 || p.nx % 2 || p.ny % 2)
    return fail(nullptr, FCNS_EINVAL, "nx and ny must be even and >= 4");
  if (p.fc_d < 2 || p.fc_C < 1 || p.nz < 2 * p.fc_d)
    return fail(nullptr, FCNS_EINVAL, "need d >= 2, C >= 1 and nz >= 2d");
  if ((p.nz + p.fc_C) % 2) return fail(nullptr, FCNS_EINVAL, "nz + C must be even");
  if (!(p.lx > 0 && p.ly > 0 && p.lz > 0)) return fail(nullptr, FCNS_EINVAL, "box lengths must be > 0");
  if (p.rk_order < 1 || p.rk_order > 4) return fail(nullptr, FCNS_EINVAL, "rk_order must be 1..4");
  if (p.precision != FCNS_FP64 && p.precision != FCNS_MIXED)
    return fail(nullptr, FCNS_EINVAL, "precision must be FCNS_FP64 or FCNS_MIXED");
  if (!p.fc_table) return fail(nullptr, FCNS_EINVAL, "fc_table is NULL");
  if (p.nx > 512 || p.ny > 1024) return fail(nullptr, FCNS_EINVAL, "need nx <= 512 and ny <= 1024");
  const int npr = p.nz + p.fc_C;
  if (npr > z_max_npr()) return fail(nullptr, FCNS_EINVAL, "N' = nz + C must be <= 512");

  fcns_ctx* c = new fcns_ctx();
  c->prob = p;
  c->prob.fc_table = nullptr;
  c->stream = (hipStream_t)hip_stream;
  c->nf = p.boussinesq ? 4 : 3;
  c->mixed = p.precision == FCNS_MIXED;
  Geom& g = c->g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.nkx = p.nx / 2 + 1;
  g.nkxp = (g.nkx + 3) / 4 * 4;
  g.npr = npr;
  g.C = p.fc_C;
  g.d = p.fc_d;
  g.npen = (long long)g.nkxp * g.ny;
  g.lx = p.lx;
  g.ly = p.ly;
  g.lz = p.lz;
  g.dz = p.lz / (p.nz - 1);
  g.lzp = npr * g.dz;
  g.kxs = 2.0 * M_PI / p.lx;
  g.kys = 2.0 * M_PI / p.ly;
  g.kzs = 2.0 * M_PI / g.lzp;

  std::vector<cpx<double>> twz, twx, twy;
  if (!make_plan_order(npr, z_radices(npr), c->plz, c->big_z, twz) || !make_plan(p.nx, c->plx, c->big_x, twx) ||
      !make_plan(p.ny, c->ply, c->big_y, twy)) {
    delete c;
    return fail(nullptr, FCNS_EINVAL, "unsupported transform length (more than 12 radix stages)");
  }
  if (y_lds_bytes(p.ny, c->ply.tsize, sizeof(cpx<double>)) > 160 * 1024) {
    delete c;
    return fail(nullptr, FCNS_EINVAL, "ny too large for the y pass (its lines must fit in LDS)");
  }

  // M_r = A_r Q_r^T in extended precision (App. B)
  const int d = p.fc_d, C = p.fc_C;
  const double* Qr = p.fc_table;
  const double* Ar = p.fc_table + d * d;
  c->hostM.resize((size_t)C * d);
  for (int i = 0; i < C; ++i)
    for (int j = 0; j < d; ++j) {
      long double acc = 0.0L;
      for (int k = 0; k < d; ++k) acc += (long double)Ar[i * d + k] * (long double)Qr[j * d + k];
      c->hostM[(size_t)i * d + j] = (double)acc;
    }

  const double beta = p.filter_beta > 0 ? p.filter_beta : 16.0 * log(10.0);
  const double two_p = p.filter_2p > 0 ? p.filter_2p : 100.0;
  c->prob.filter_beta = beta;
  c->prob.filter_2p = two_p;
  auto rz = roots(npr);
  auto sx = filter_table(p.nx, g.nkx, true, beta, two_p);
  auto sy = filter_table(p.ny, p.ny, false, beta, two_p);
  auto sz = filter_table(npr, npr, false, beta, two_p);
  auto to_f32 = [](const std::vector<cpx<double>>& t) {
    std::vector<cpx<float>> o(t.size());
    for (size_t i = 0; i < t.size(); ++i) o[i] = mk((float)t[i].x, (float)t[i].y);
    return o;
  };
  fcns_status st = FCNS_OK;
  if (c->mixed) {
    auto fz = to_f32(twz), fx = to_f32(twx), fy = to_f32(twy);
    if ((st = upload(c, &c->twz_f, fz.data(), fz.size())) ||
        (st = upload(c, &c->twx_f, fx.data(), fx.size())) ||
        (st = upload(c, &c->twy_f, fy.data(), fy.size()))) {
      g_create_err = c->err;
      free_all(c);
      delete c;
      return st;
    }
  }
  if ((st = upload(c, &c->twz, twz.data(), twz.size())) ||
      (st = upload(c, &c->twx, twx.data(), twx.size())) ||
      (st = upload(c, &c->twy, twy.data(), twy.size())) ||
      (st = upload(c, &c->rootz, rz.data(), rz.size())) ||
      (st = upload(c, &c->fcM, c->hostM.data(), c->hostM.size())) ||
      (st = upload(c, &c->sigx, sx.data(), sx.size())) ||
      (st = upload(c, &c->sigy, sy.data(), sy.size())) ||
      (st = upload(c, &c->sigz, sz.data(), sz.size()))) {
    g_create_err = c->err;
    free_all(c);
    delete c;
    return st;
  }
  c->S = (long long)npr * g.npen;
  c->M = (long long)p.nz * g.npen;
  const int nf = c->nf;
  if ((st = alloc(c, &c->P, nf * c->S)) || (st = alloc(c, &c->Q, nf * c->S)) ||
      (st = alloc(c, &c->VS, nf * c->S)) || (st = alloc(c, &c->MV, 2 * nf * c->M)) ||
      (st = alloc(c, &c->MVT, 2 * nf * c->M)) || (st = alloc(c, &c->XYB, 3 * nf * c->M)) ||
      (st = alloc(c, &c->NLB, nf * c->M)) || (st = alloc(c, &c->PM, c->M)) ||
      (st = alloc(c, &c->GW, 4 * g.npen)) || (st = alloc(c, &c->GWT, 4 * g.npen)) ||
      (st = hipMalloc((void**)&c->DG, sizeof(double) * (5 * (size_t)p.nz + g.nkx + p.ny)) ==
                    hipSuccess ? FCNS_OK : fail(c, FCNS_ENOMEM, "device allocation failed")) ||
      (st = hipHostMalloc((void**)&c->hflag, sizeof(cpx<double>),
                          hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess
                ? FCNS_OK : fail(c, FCNS_ENOMEM, "pinned host allocation failed")) ||
      (st = check_hip(c, hipHostGetDevicePointer((void**)&c->dflag, c->hflag, 0),
                      "flag device address"))) {
    g_create_err = c->err;
    free_all(c);
    delete c;
    return st;
  }
  launch_fill(c->GW, 4 * g.npen, c->stream);
  *(volatile int*)c->hflag = 0;
  launch_fill(reinterpret_cast<cpx<double>*>(c->dflag), 1, c->stream);
  if ((st = check_launch(c, "fill")) != FCNS_OK) {
    g_create_err = c->err;
    free_all(c);
    delete c;
    return st;
  }
  *out = c;
  return FCNS_OK;
}

extern "C" fcns_status fcns_destroy(fcns_ctx* c) {
  if (!c) return FCNS_OK;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return FCNS_OK;
}

extern "C" const char* fcns_last_error(const fcns_ctx* c) {
  return c ? c->err.c_str() : g_create_err.c_str();
}

extern "C" int32_t fcns_npr(const fcns_ctx* c) { return c ? c->g.npr : 0; }

extern "C" fcns_status fcns_footprint(const fcns_problem* p, int64_t* bytes) {
  if (!p || !bytes) return FCNS_EINVAL;
  if (p->nx < 4 || p->ny < 4 || p->nz < 2 || p->fc_C < 1) return FCNS_EINVAL;
  const long long nkxp = ((long long)p->nx / 2 + 1 + 3) / 4 * 4;
  const long long npen = nkxp * p->ny;
  const long long S = (long long)(p->nz + p->fc_C) * npen, M = (long long)p->nz * npen;
  const long long nf = p->boussinesq ? 4 : 3;
  // P, Q, VS; MV, MVT, XYB, NLB, PM; GW, GWT (complex128), plus tables
  const long long elems = 3 * nf * S + (2 * nf + 2 * nf + 3 * nf + nf + 1) * M + 8 * npen;
  const long long tables = 16LL * (4LL * (p->nx + p->ny + p->nz + p->fc_C) + 4096) +
                           8LL * p->fc_C * p->fc_d;
  *bytes = (int64_t)(elems * 16 + tables);
  return FCNS_OK;
}

extern "C" fcns_status fcns_set_params(fcns_ctx* c, double nu, double kappa, double gamma,
                                       double forcing_x) {
  if (!c) return FCNS_EINVAL;
  if (!(nu >= 0.0) || !(kappa >= 0.0) || !std::isfinite(gamma) || !std::isfinite(forcing_x))
    return fail(c, FCNS_EINVAL, "need nu, kappa >= 0 and finite gamma, forcing_x");
  c->prob.nu = nu;
  c->prob.kappa = kappa;
  c->prob.gamma = gamma;
  c->prob.forcing_x = forcing_x;
  return FCNS_OK;
}

extern "C" void* fcns_stream(const fcns_ctx* c) { return c ? (void*)c->stream : nullptr; }

// ---------------------------------------------------------------- pieces
// physical fields (nfields consecutive [nz][ny][nx] arrays) -> mixed (kx, ky, z)
static void phys_to_mixed(fcns_ctx* c, const double* phys, int nfields, cpx<double>* mixed) {
  const Geom& g = c->g;
  const long long pfs = (long long)g.nz * g.ny * g.nx;
  launch_x_r2c(xargs(c), c->big_x, phys, mixed, pfs, c->M, (long long)g.nz * g.ny, nfields,
               c->stream);
  launch_y<double>(yargs(c), c->big_y, false, 0, mixed, mixed, nullptr, c->M, c->M, g.nz, nfields,
           c->stream);
}

// mixed (kx, ky, z) fields at stride mstride -> physical; scratch: XYB
static void mixed_to_phys(fcns_ctx* c, const cpx<double>* mixed, long long mstride, int nfields,
                          double* phys, int nplanes) {
  const Geom& g = c->g;
  const long long plane = (long long)g.ny * g.nkxp;
  const long long xfs = (long long)nplanes * plane;
  launch_y<double>(yargs(c), c->big_y, true, 0, mixed, c->XYB, nullptr, mstride, xfs, nplanes, nfields,
           c->stream);
  launch_x_c2r(xargs(c), c->big_x, c->XYB, phys, xfs, (long long)nplanes * g.ny * g.nx,
               (long long)nplanes * g.ny, nfields, c->stream);
}

// nonlinear term of the fields whose mixed v_f, dv_f/dz are in mv (slots 2f,
// 2f+1) into NLB (mixed if fwd_y, else (kx, y, z)); T is the transform and
// storage type of MV / XYB / NLB.
template <typename T>
static void nonlinear_from_mixed(fcns_ctx* c, const cpx<T>* mv, int nfields, bool fwd_y) {
  const Geom& g = c->g;
  const long long M = c->M;
  const bool f32 = sizeof(T) == sizeof(float);
  cpx<T>* xyb = reinterpret_cast<cpx<T>*>(c->XYB);
  cpx<T>* nlb = reinterpret_cast<cpx<T>*>(c->NLB);
  // y back transforms into XYB (blocked when the x pass reads that layout)
  XArgs xa = xargs(c, f32);
  xa.blk_in = (c->xyblk && x_reads_blocked(xa)) ? 1 : 0;
  YArgs yb1 = yargs(c, f32, true), yb0 = yargs(c, f32);
  yb1.blk = yb0.blk = xa.blk_in ? 2 : 0;
  if (fwd_y && c->slab > 0 && c->slab < g.nz) {
    // slab by slab: the (kx, y, z) intermediates of a slab of planes are
    // written and read back within its four launches, in the first part of
    // XYB (4 nf slab fields), soon after they are written (the last ones
    // still in the caches); only the mixed nonlinear term reaches NLB
    const long long P = (long long)g.ny * g.nkxp;
    const long long Ms = (long long)c->slab * P;
    cpx<T>* nls = xyb + 3 * nfields * Ms;
    tbeg(c, T_XYSLAB);
    for (int z0 = 0; z0 < g.nz; z0 += c->slab) {
      const int nzs = std::min(c->slab, g.nz - z0);
      const long long off = (long long)z0 * P;
      launch_y<T>(yb1, c->big_y, true, 1, mv + off, xyb, xyb + Ms, 2 * M, 3 * Ms, nzs, nfields,
                  c->stream);
      launch_y<T>(yb0, c->big_y, true, 0, mv + M + off, xyb + 2 * Ms, nullptr, 2 * M, 3 * Ms,
                  nzs, nfields, c->stream);
      launch_x_nl<T>(xa, c->big_x, xyb, nls, Ms, (long long)nzs * g.ny, nfields, c->stream);
      launch_y<T>(yargs(c, f32), c->big_y, false, 0, nls, nlb + off, nullptr, Ms, M, nzs,
                  nfields, c->stream);
    }
    tend(c);
    return;
  }
  tbeg(c, T_YBACK_DY);
  launch_y<T>(yb1, c->big_y, true, 1, mv, xyb, xyb + M, 2 * M, 3 * M, g.nz, nfields, c->stream);
  tend(c);
  tbeg(c, T_YBACK_DZ);
  launch_y<T>(yb0, c->big_y, true, 0, mv + M, xyb + 2 * M, nullptr, 2 * M, 3 * M, g.nz, nfields,
              c->stream);
  tend(c);
  tbeg(c, T_XNL);
  launch_x_nl<T>(xa, c->big_x, xyb, nlb, M, (long long)g.nz * g.ny, nfields, c->stream);
  tend(c);
  if (fwd_y) {
    tbeg(c, T_YFWD);
    launch_y<T>(yargs(c, f32), c->big_y, false, 0, nlb, nlb, nullptr, M, M, g.nz, nfields,
                c->stream);
    tend(c);
  }
}

// the mixed v, dv/dz of the continued state src into MV, in the type the
// rk_step pipeline reads (FP32 for a mixed-precision context); check: the
// transform also raises the context's non-finite flag
static void state_to_mv(fcns_ctx* c, const cpx<double>* src, bool check = false) {
  ZArgs a = zargs(c, c->mixed);
  if (check) a.nonfinite = c->dflag;
  if (c->mixed) {
    cpx<float>* mv = reinterpret_cast<cpx<float>*>(c->MV);
    launch_z_back<float>(a, c->big_z, src, mv, mv + c->M, c->S, 2 * c->M, c->nf, c->stream);
  } else {
    launch_z_back<double>(a, c->big_z, src, c->MV, c->MV + c->M, c->S, 2 * c->M, c->nf,
                          c->stream);
  }
}

static int read_flag(const fcns_ctx* c) { return *(volatile const int*)c->hflag; }

// a new state: the flag cleared when the stream gets there
static void clear_flag(fcns_ctx* c) {
  launch_fill(reinterpret_cast<cpx<double>*>(c->dflag), 1, c->stream);
}

// After the steps of one call: in the synchronous mode wait for them and
// report a non-finite state.
static fcns_status finish_steps(fcns_ctx* c, const char* what) {
  fcns_status st = check_launch(c, what);
  if (st != FCNS_OK || c->check_mode != FCNS_CHECK_SYNC) return st;
  if ((st = check_hip(c, hipStreamSynchronize(c->stream), what))) return st;
  if (read_flag(c)) return fail(c, FCNS_ENONFINITE, "non-finite value in the state after a step");
  return FCNS_OK;
}

// ---------------------------------------------------------------- entry points
extern "C" fcns_status fcns_fc_extend(fcns_ctx* c, const double* in, int64_t nlines, int64_t in_ps,
                                      int64_t in_ls, double* out, int64_t out_ps, int64_t out_ls) {
  if (!c) return FCNS_EINVAL;
  if (nlines < 0) return fail(c, FCNS_EINVAL, "nlines < 0");
  if (nlines == 0) return FCNS_OK;
  if (!in || !out) return fail(c, FCNS_EINVAL, "NULL pointer");
  launch_fc_extend(in, nlines, in_ps, in_ls, out, out_ps, out_ls, c->g.nz, c->g.C, c->g.d, c->fcM,
                   c->stream);
  return check_launch(c, "fc_extend");
}

extern "C" fcns_status fcns_fc_derivative(fcns_ctx* c, int32_t order, const double* in,
                                          int64_t nlines, int64_t ps, int64_t ls, double* out) {
  if (!c) return FCNS_EINVAL;
  if (order != 1 && order != 2) return fail(c, FCNS_EINVAL, "order must be 1 or 2");
  if (nlines < 0) return fail(c, FCNS_EINVAL, "nlines < 0");
  if (nlines == 0) return FCNS_OK;
  if (!in || !out) return fail(c, FCNS_EINVAL, "NULL pointer");
  launch_fc_derivative(zargs(c), c->big_z, in, out, nlines, ps, ls, order, c->stream);
  return check_launch(c, "fc_derivative");
}


// continued spectral state of `nfields` mixed fields (stride M) into dst
// (stride S), then the mixed v, dv/dz of the state into mv (slots 2f, 2f+1)
static void mixed_to_state(fcns_ctx* c, const cpx<double>* mixed, int nfields, cpx<double>* dst,
                           cpx<double>* mv) {
  launch_z_fwd(zargs(c), c->big_z, mixed, dst, c->M, c->S, nfields, 0, c->stream);
  if (mv)
    launch_z_back<double>(zargs(c), c->big_z, dst, mv, mv + c->M, c->S, 2 * c->M, nfields,
                          c->stream);
}

extern "C" fcns_status fcns_set_state(fcns_ctx* c, const double* v, const double* theta) {
  if (!c) return FCNS_EINVAL;
  if (!v) return fail(c, FCNS_EINVAL, "v is NULL");
  if (c->prob.boussinesq && !theta) return fail(c, FCNS_EINVAL, "theta required (Boussinesq)");
  phys_to_mixed(c, v, 3, c->XYB);
  if (c->nf == 4) phys_to_mixed(c, theta, 1, c->XYB + 3 * c->M);
  mixed_to_state(c, c->XYB, c->nf, c->P, nullptr);
  state_to_mv(c, c->P);
  launch_fill(c->GW, 4 * c->g.npen, c->stream);
  clear_flag(c);
  fcns_status st = check_launch(c, "set_state");
  if (st == FCNS_OK) {
    c->has_state = true;
    c->has_pressure = false;
  }
  return st;
}

// The z pass of one stage (Sec. 4.4 steps 1-5 after the nonlinear term is in
// NLB): W the previous stage's state, OUT the new one, cj the stage
// coefficient, pressure: keep the mixed pressure.  fused: one kernel for the
// whole pass (FP64, OUT != W, N' <= 288), else stage A, stage B and the back
// transform of the new state.  T as in rk_stage.
template <typename T>
static void z_part_args(const fcns_ctx* c, cpx<double>* W, cpx<double>* OUT, double cj,
                        bool pressure, bool fused, StageAArgs& A, StageBArgs& B) {
  const cpx<T>* mv = reinterpret_cast<const cpx<T>*>(c->MV);
  const cpx<T>* nlb = reinterpret_cast<const cpx<T>*>(c->NLB);
  const Geom& g = c->g;
  const long long S = c->S, M = c->M;
  const int nf = c->nf;
  memset(&A, 0, sizeof(A));
  for (int f = 0; f < nf; ++f) {
    A.nl[f] = nlb + f * M;
    A.vt[f] = c->P + f * S;
    A.w[f] = W + f * S;
    A.out[f] = (f < 3 && !fused) ? c->VS + f * S : OUT + f * S;
    A.buoy[f] = nullptr;
  }
  if (nf == 4) {
    if (fused) {
      A.buoy[2] = W + 3 * S;  // continued theta of the previous stage (for w)
      A.buoy[3] = W + 2 * S;  // continued w of the previous stage (for theta)
    } else {
      A.buoy[2] = mv + (2 * 3) * M;  // mixed theta of the previous stage
      A.buoy[3] = mv + (2 * 2) * M;  // mixed w of the previous stage
    }
  }
  A.gwall = c->GW;
  A.c = cj;
  A.nu = c->prob.nu;
  A.kappa = c->prob.kappa;
  A.gamma = c->prob.gamma;
  A.forcing_sum = c->prob.forcing_x * (double)g.nx * (double)g.ny;
  memset(&B, 0, sizeof(B));
  for (int i = 0; i < 3; ++i) {
    B.vs[i] = fused ? OUT + i * S : c->VS + i * S;
    B.vout[i] = OUT + i * S;
  }
  B.gwall = c->GW;
  B.pmix = pressure ? c->PM : nullptr;
  B.c = cj;
}

template <typename T>
static void z_part(fcns_ctx* c, cpx<double>* W, cpx<double>* OUT, double cj, bool pressure,
                   bool fused) {
  const long long M = c->M;
  const int nf = c->nf;
  StageAArgs A;
  StageBArgs B;
  z_part_args<T>(c, W, OUT, cj, pressure, fused, A, B);
  if (fused) {
    // V* lives in OUT's velocity slots between its stage A and its
    // projection, inside one workgroup
    ZBackArgs Z{c->MV, M};
    ZArgs za = zargs(c);
    za.nonfinite = c->dflag;
    tbeg(c, T_ZPASS);
    launch_z_pass(za, c->big_z, A, B, Z, nf, c->stream);
    tend(c);
    return;
  }
  // stage A: pressureless update, wall injection, FC re-extension
  tbeg(c, T_ZSTAGEA);
  launch_z_stageA<T>(zargs(c), c->big_z, A, nf, c->stream);
  tend(c);
  // stage B: projection, next-stage wall gradient
  tbeg(c, T_ZSTAGEB);
  launch_z_stageB(zargs(c), c->big_z, B, c->stream);
  tend(c);
  // mixed v_f, dv_f/dz of the new state for the next stage's x/y passes,
  // with the non-finite check of the state
  tbeg(c, T_ZBACK);
  state_to_mv(c, OUT, true);
  tend(c);
}

static bool can_fuse(const fcns_ctx* c) { return !c->mixed && z_pass_fits(zargs(c)); }

// One RK stage j of o (Sec. 4.4), c = dt/(o-j+1).  T: type of the transforms
// and arrays of the nonlinear term (float in a mixed-precision context); the
// continued state, the FC extension, stage A's transforms of the RK combine,
// and the projection are FP64 throughout.
template <typename T>
static void rk_stage(fcns_ctx* c, int j, int o, double dt) {
  const double cj = dt / (double)(o - j + 1);
  cpx<double>* W = (j == 1) ? c->P : c->Q;
  cpx<double>* OUT = (j == o) ? c->P : c->Q;
  // y-back, x-pass with products, y-fwd: nonlinear term in mixed space
  nonlinear_from_mixed<T>(c, reinterpret_cast<const cpx<T>*>(c->MV), c->nf, true);
  const bool fused = c->zfuse && OUT != W && can_fuse(c);
  z_part<T>(c, W, OUT, cj, c->prob.keep_pressure && j == o, fused);
}

extern "C" fcns_status fcns_rk_step(fcns_ctx* c, double dt, int32_t nsteps) {
  if (!c) return FCNS_EINVAL;
  if (!c->has_state) return fail(c, FCNS_ESTATE, "rk_step before set_state");
  if (!(dt > 0.0) || nsteps < 0) return fail(c, FCNS_EINVAL, "need dt > 0 and nsteps >= 0");
  const int o = c->prob.rk_order;
  for (int n = 0; n < nsteps; ++n)
    for (int j = 1; j <= o; ++j) {
      if (c->mixed)
        rk_stage<float>(c, j, o, dt);
      else
        rk_stage<double>(c, j, o, dt);
    }
  if (nsteps > 0 && c->prob.keep_pressure) c->has_pressure = true;
  return finish_steps(c, "rk_step");
}

// A captured step (fcns_rk_graph) holds the launch choices it was captured
// with: a change of choices drops it, and the next fcns_rk_graph captures
// the step again.
static void drop_graph(fcns_ctx* c) {
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
}

extern "C" fcns_status fcns_set_y_lines(fcns_ctx* c, int32_t lines) {
  if (!c) return FCNS_EINVAL;
  if (lines != 4 && lines != 8) return fail(c, FCNS_EINVAL, "y tiles have 4 or 8 lines");
  if (lines == 8 && !y_wide_tiles(yargs(c)))
    return fail(c, FCNS_EINVAL, "8-line y tiles need ny = 512");
  c->ylines = c->ylines1 = lines;
  drop_graph(c);
  return FCNS_OK;
}

extern "C" fcns_status fcns_set_blocked(fcns_ctx* c, int32_t on) {
  if (!c) return FCNS_EINVAL;
  if (on && !x_reads_blocked(xargs(c)))
    return fail(c, FCNS_EINVAL, "the blocked layout needs the wave-level x pass (nx = 256, 512)");
  c->xyblk = on != 0;
  drop_graph(c);
  return FCNS_OK;
}

extern "C" fcns_status fcns_set_slab(fcns_ctx* c, int32_t planes) {
  if (!c) return FCNS_EINVAL;
  if (planes < 0) return fail(c, FCNS_EINVAL, "slab planes must be >= 0");
  // the slab scratch (4 nf slab fields) lives in XYB (3 nf whole fields)
  if (planes > 0 && 4LL * planes > 3LL * c->g.nz)
    return fail(c, FCNS_EINVAL, "slab larger than 3/4 of the planes");
  c->slab = planes;
  drop_graph(c);
  return FCNS_OK;
}

extern "C" fcns_status fcns_set_z_fused(fcns_ctx* c, int32_t on) {
  if (!c) return FCNS_EINVAL;
  if (on && !can_fuse(c))
    return fail(c, FCNS_EINVAL, "the fused z pass needs an FP64 context and N' <= 288");
  c->zfuse = on != 0;
  drop_graph(c);
  return FCNS_OK;
}

extern "C" fcns_status fcns_set_finite_check(fcns_ctx* c, int32_t mode) {
  if (!c) return FCNS_EINVAL;
  if (mode != FCNS_CHECK_OFF && mode != FCNS_CHECK_SYNC && mode != FCNS_CHECK_DEFERRED)
    return fail(c, FCNS_EINVAL, "unknown check mode");
  c->check_mode = mode;
  return FCNS_OK;
}

extern "C" fcns_status fcns_check_finite(fcns_ctx* c) {
  if (!c) return FCNS_EINVAL;
  fcns_status st = check_hip(c, hipStreamSynchronize(c->stream), "check_finite");
  if (st != FCNS_OK) return st;
  if (read_flag(c)) return fail(c, FCNS_ENONFINITE, "non-finite value in the state after a step");
  return FCNS_OK;
}

extern "C" int32_t fcns_nonfinite_flag(const fcns_ctx* c) {
  return (c && c->hflag) ? read_flag(c) : 0;
}

// Capture one step (all o stages) for this dt on a private stream; the graph
// is replayed on the context stream.  The captured kernels are exactly those
// of fcns_rk_step (no memory-set nodes: buffers are cleared by kernels).
static fcns_status capture_step(fcns_ctx* c, double dt) {
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  fcns_status st;
  if (!c->cap_stream &&
      (st = check_hip(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking),
                      "graph stream")))
    return st;
  // the captured work must follow what is already queued on the context stream
  if ((st = check_hip(c, hipStreamSynchronize(c->stream), "graph capture"))) return st;
  hipStream_t saved = c->stream;
  const bool timing = c->timing;
  c->timing = false;
  c->stream = c->cap_stream;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const int o = c->prob.rk_order;
    for (int j = 1; j <= o; ++j) {
      if (c->mixed)
        rk_stage<float>(c, j, o, dt);
      else
        rk_stage<double>(c, j, o, dt);
    }
    const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    e = (e2 != hipSuccess) ? e2 : hipGetLastError();
  }
  c->stream = saved;
  c->timing = timing;
  if (e == hipSuccess) e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->graph = nullptr;
    return check_hip(c, e, "graph capture");
  }
  c->graph_dt = dt;
  return FCNS_OK;
}

extern "C" fcns_status fcns_rk_graph(fcns_ctx* c, double dt, int32_t nsteps) {
  if (!c) return FCNS_EINVAL;
  if (!c->has_state) return fail(c, FCNS_ESTATE, "rk_graph before set_state");
  if (!(dt > 0.0) || nsteps < 0) return fail(c, FCNS_EINVAL, "need dt > 0 and nsteps >= 0");
  fcns_status st;
  if ((!c->graph || c->graph_dt != dt) && (st = capture_step(c, dt))) return st;
  for (int n = 0; n < nsteps; ++n)
    if ((st = check_hip(c, hipGraphLaunch(c->graph, c->stream), "graph launch"))) return st;
  if (nsteps > 0 && c->prob.keep_pressure) c->has_pressure = true;
  return finish_steps(c, "rk_graph");
}

// ---------------------------------------------------------------- autotuner
// Mean duration (ms) of `reps` runs of f on the context stream.
template <typename F>
static float time_ms(fcns_ctx* c, F&& f, int reps) {
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  f();  // warm-up (also the first-use LDS opt-in)
  (void)hipEventRecord(a, c->stream);
  for (int i = 0; i < reps; ++i) f();
  (void)hipEventRecord(b, c->stream);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

static fcns_status set_z_plan(fcns_ctx* c, const std::vector<int>& rs) {
  FFTPlan pl;
  bool big;
  std::vector<cpx<double>> t;
  if (!make_plan_order(c->g.npr, rs, pl, big, t)) return fail(c, FCNS_EINVAL, "bad z plan");
  cpx<double>* d = nullptr;
  cpx<float>* f = nullptr;
  fcns_status st;
  if ((st = upload(c, &d, t.data(), t.size()))) return st;
  if (c->mixed) {
    std::vector<cpx<float>> tf(t.size());
    for (size_t i = 0; i < t.size(); ++i) tf[i] = mk((float)t[i].x, (float)t[i].y);
    if ((st = upload(c, &f, tf.data(), tf.size()))) {
      (void)hipFree(d);
      return st;
    }
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(c->twz);
  if (c->twz_f) (void)hipFree(c->twz_f);
  c->twz = d;
  c->twz_f = f;
  c->plz = pl;
  c->big_z = big;
  drop_graph(c);   // a captured step holds the old tables
  return FCNS_OK;
}

extern "C" fcns_status fcns_autotune(fcns_ctx* c, char* report, int32_t report_len) {
  if (!c) return FCNS_EINVAL;
  if (!c->has_state) return fail(c, FCNS_ESTATE, "autotune before set_state");
  const Geom& g = c->g;
  const long long M = c->M;
  const int nf = c->nf, reps = 3;
  const bool f32 = c->mixed;
  std::string rep;
  char line[256];
  // the timed trials carry no kernel-timing events
  const bool timing = c->timing;
  c->timing = false;
  // y pass: persistent grid size and prefetch, chosen separately for the back
  // transform with d/dy (two transforms per tile) and for the two launches of
  // one transform per tile (back of dv/dz, forward of NL), on the state's
  // fields
  {
    auto pass_dy = [&](auto* mv, auto* xy, bool f) {
      launch_y(yargs(c, f, true), c->big_y, true, 1, mv, xy, xy + M, 2 * M, 3 * M, g.nz, nf,
               c->stream);
    };
    auto pass_one = [&](auto* mv, auto* xy, auto* nlb, bool f) {
      launch_y(yargs(c, f), c->big_y, true, 0, mv + M, xy + 2 * M, decltype(xy)(nullptr), 2 * M,
               3 * M, g.nz, nf, c->stream);
      launch_y(yargs(c, f), c->big_y, false, 0, nlb, nlb, decltype(xy)(nullptr), M, M, g.nz, nf,
               c->stream);
    };
    float best1 = 1e30f, best0 = 1e30f;
    long long bg1 = Y_GRID, bg0 = Y_GRID;
    int bpf1 = 0, bpf0 = 0, bl1 = 4, bl0 = 4;
    const bool wide = y_wide_tiles(yargs(c));
    for (int lines : {4, 8})
    for (int nopf : {0, 1})
      for (long long gsz : {256LL, 512LL, 1024LL, 2048LL, 4096LL}) {
        if (lines == 8 && !wide) continue;
        c->ygrid = c->ygrid1 = gsz;
        c->ynopf = c->ynopf1 = nopf;
        c->ylines = c->ylines1 = lines;
        const float ms1 = time_ms(c, [&] {
          if (f32)
            pass_dy(reinterpret_cast<cpx<float>*>(c->MV), reinterpret_cast<cpx<float>*>(c->XYB),
                    true);
          else
            pass_dy(c->MV, c->XYB, false);
        }, reps);
        const float ms0 = time_ms(c, [&] {
          if (f32)
            pass_one(reinterpret_cast<cpx<float>*>(c->MV), reinterpret_cast<cpx<float>*>(c->XYB),
                     reinterpret_cast<cpx<float>*>(c->NLB), true);
          else
            pass_one(c->MV, c->XYB, c->NLB, false);
        }, reps);
        if (ms1 < best1) {
          best1 = ms1;
          bg1 = gsz;
          bpf1 = nopf;
          bl1 = lines;
        }
        if (ms0 < best0) {
          best0 = ms0;
          bg0 = gsz;
          bpf0 = nopf;
          bl0 = lines;
        }
      }
    c->ygrid1 = bg1;
    c->ynopf1 = bpf1;
    c->ylines1 = bl1;
    c->ygrid = bg0;
    c->ynopf = bpf0;
    c->ylines = bl0;
    snprintf(line, sizeof(line),
             "y: grid %lld%s, %d lines (%.3f ms), with d/dy %lld%s, %d lines (%.3f ms); ", bg0,
             bpf0 ? " no-prefetch" : "", bl0, best0, bg1, bpf1 ? " no-prefetch" : "", bl1, best1);
    rep += line;
  }
  // x pass with products: kernel variant (inputs: the y pass just run)
  {
    float best = 1e30f;
    int bv = 0;
    for (int v : {0, 1, 2, 3}) {
      if ((v == 2 && g.nx > 512) || (v == 3 && g.nx > 256)) continue;
      c->xvar = v;
      const float ms = time_ms(c, [&] {
        if (f32)
          launch_x_nl<float>(xargs(c, true), c->big_x, reinterpret_cast<cpx<float>*>(c->XYB),
                             reinterpret_cast<cpx<float>*>(c->NLB), M, (long long)g.nz * g.ny,
                             nf, c->stream);
        else
          launch_x_nl<double>(xargs(c), c->big_x, c->XYB, c->NLB, M, (long long)g.nz * g.ny, nf,
                              c->stream);
      }, reps);
      if (ms < best) {
        best = ms;
        bv = v;
      }
    }
    c->xvar = bv;
    snprintf(line, sizeof(line), "x: variant %d (%.3f ms); ", bv, best);
    rep += line;
  }
  // y and x passes over whole arrays or slab by slab (timed on the state's
  // mixed fields; XYB and NLB are scratch)
  {
    float best = 1e30f;
    int bs = 0;
    bool bb = false;
    for (int blk : {0, 1}) {
      if (blk && !x_reads_blocked(xargs(c))) continue;
      for (int sl : {0, 16, 32, 48, 64, 96, 128}) {
        if (sl > 0 && (sl >= g.nz || 4 * sl > 3 * g.nz)) continue;
        c->slab = sl;
        c->xyblk = blk != 0;
        const float ms = time_ms(c, [&] {
          if (f32)
            nonlinear_from_mixed<float>(c, reinterpret_cast<const cpx<float>*>(c->MV), nf, true);
          else
            nonlinear_from_mixed<double>(c, c->MV, nf, true);
        }, reps);
        if (ms < best) {
          best = ms;
          bs = sl;
          bb = blk != 0;
        }
      }
    }
    c->slab = bs;
    c->xyblk = bb;
    snprintf(line, sizeof(line), "y/x: %s, %s (%.3f ms); ",
             bb ? "blocked intermediates" : "row-major intermediates",
             bs > 0 ? ("slabs of " + std::to_string(bs) + " planes").c_str() : "whole arrays",
             best);
    rep += line;
  }
  // z: radix order of a run-time plan, timed on the back-transform of the
  // state (a compiled plan, when the length has one, is kept)
  {
    std::vector<int> rs = z_radices(g.npr);
    const bool compiled = g.npr == 288 && rs == std::vector<int>{16, 18};
    std::vector<int> best_rs = rs;
    float best = 1e30f;
    if (!compiled) {
      std::vector<int> perm = rs;
      std::sort(perm.begin(), perm.end());
      int n = 0;
      do {
        fcns_status st = set_z_plan(c, perm);
        if (st) {
          c->timing = timing;
          return st;
        }
        const float ms = time_ms(c, [&] {
          launch_z_back<double>(zargs(c), c->big_z, c->P, c->MVT, c->MVT + M, c->S, 2 * M, nf,
                                c->stream);
        }, reps);
        if (ms < best) {
          best = ms;
          best_rs = perm;
        }
      } while (++n < 24 && std::next_permutation(perm.begin(), perm.end()));
      fcns_status st = set_z_plan(c, best_rs);
      if (st) {
        c->timing = timing;
        return st;
      }
    }
    rep += "z: radices";
    for (int r : best_rs) rep += " " + std::to_string(r);
    if (compiled) {
      rep += " (compiled plan)";
    } else {
      snprintf(line, sizeof(line), " (%.3f ms)", best);
      rep += line;
    }
  }
  // z pass: one fused kernel or the three separate ones, timed as a first
  // stage would run them (the wall gradient is saved and restored; Q, VS and
  // the mixed arrays are scratch here)
  if (can_fuse(c)) {
    const size_t gwb = 4 * (size_t)g.npen * sizeof(cpx<double>);
    (void)hipMemcpyAsync(c->GWT, c->GW, gwb, hipMemcpyDeviceToDevice, c->stream);
    const double cj = 1e-3;
    const float ms_f = time_ms(c, [&] { z_part<double>(c, c->P, c->Q, cj, false, true); }, reps);
    const float ms_s = time_ms(c, [&] { z_part<double>(c, c->P, c->Q, cj, false, false); }, reps);
    (void)hipMemcpyAsync(c->GW, c->GWT, gwb, hipMemcpyDeviceToDevice, c->stream);
    c->zfuse = ms_f <= ms_s;
    snprintf(line, sizeof(line), "; z pass: %s (fused %.3f ms, split %.3f ms)",
             c->zfuse ? "fused" : "split", ms_f, ms_s);
    rep += line;
  }
  // the mixed-space fields of the state were overwritten only in scratch; the
  // ones the next step reads are rebuilt from the state
  state_to_mv(c, c->P);
  c->timing = timing;
  drop_graph(c);
  fcns_status st = check_launch(c, "autotune");
  if (report && report_len > 0) {
    strncpy(report, rep.c_str(), (size_t)report_len - 1);
    report[report_len - 1] = 0;
  }
  return st;
}

// The launch choices as "key=value" pairs separated by ';' (what
// fcns_autotune chose, or the defaults), and the inverse.
static std::string choices_string(const fcns_ctx* c) {
  std::string z;
  for (int s = 0; s < c->plz.nst; ++s) z += (s ? "." : "") + std::to_string(c->plz.r[s]);
  char buf[512];
  snprintf(buf, sizeof(buf),
           "ygrid=%lld;ynopf=%d;ylines=%d;ygrid1=%lld;ynopf1=%d;ylines1=%d;xvar=%d;slab=%d;"
           "blocked=%d;zfused=%d;zplan=%s",
           c->ygrid, c->ynopf, c->ylines, c->ygrid1, c->ynopf1, c->ylines1, c->xvar, c->slab,
           c->xyblk ? 1 : 0, c->zfuse ? 1 : 0, z.c_str());
  return buf;
}

extern "C" fcns_status fcns_get_choices(const fcns_ctx* c, char* out, int32_t len) {
  if (!c || !out || len <= 0) return FCNS_EINVAL;
  const std::string s = choices_string(c);
  if ((int32_t)s.size() >= len) return FCNS_EINVAL;
  memcpy(out, s.c_str(), s.size() + 1);
  return FCNS_OK;
}

extern "C" fcns_status fcns_set_choices(fcns_ctx* c, const char* text) {
  if (!c || !text) return FCNS_EINVAL;
  // parse and check everything before changing anything
  struct {
    long long ygrid, ygrid1;
    int ynopf, ylines, ynopf1, ylines1, xvar, slab;
    bool xyblk, zfuse;
  } t{c->ygrid, c->ygrid1, c->ynopf, c->ylines, c->ynopf1, c->ylines1, c->xvar, c->slab,
      c->xyblk, c->zfuse};
  std::vector<int> zplan;
  std::string all(text);
  size_t pos = 0;
  while (pos < all.size()) {
    size_t end = all.find(';', pos);
    if (end == std::string::npos) end = all.size();
    const std::string item = all.substr(pos, end - pos);
    pos = end + 1;
    if (item.empty()) continue;
    const size_t eq = item.find('=');
    if (eq == std::string::npos) return fail(c, FCNS_EINVAL, "choice without '=': " + item);
    const std::string k = item.substr(0, eq), v = item.substr(eq + 1);
    char* e = nullptr;
    if (k == "zplan") {
      size_t q = 0;
      while (q < v.size()) {
        size_t d = v.find('.', q);
        if (d == std::string::npos) d = v.size();
        zplan.push_back(atoi(v.substr(q, d - q).c_str()));
        q = d + 1;
      }
      continue;
    }
    const long long x = strtoll(v.c_str(), &e, 10);
    if (v.empty() || *e) return fail(c, FCNS_EINVAL, "bad value: " + item);
    if (k == "ygrid") t.ygrid = x;
    else if (k == "ynopf") t.ynopf = (int)x;
    else if (k == "ylines") t.ylines = (int)x;
    else if (k == "ygrid1") t.ygrid1 = x;
    else if (k == "ynopf1") t.ynopf1 = (int)x;
    else if (k == "ylines1") t.ylines1 = (int)x;
    else if (k == "xvar") t.xvar = (int)x;
    else if (k == "slab") t.slab = (int)x;
    else if (k == "blocked") t.xyblk = x != 0;
    else if (k == "zfused") t.zfuse = x != 0;
    else return fail(c, FCNS_EINVAL, "unknown choice: " + k);
  }
  const YArgs ya = yargs(c);
  XArgs xa = xargs(c);
  xa.variant = t.xvar;
  if (t.ygrid < 0 || t.ygrid1 < 0 || t.ygrid > (1 << 20) || t.ygrid1 > (1 << 20) ||
      (t.ylines != 4 && t.ylines != 8) || (t.ylines1 != 4 && t.ylines1 != 8) ||
      ((t.ylines == 8 || t.ylines1 == 8) && !y_wide_tiles(ya)) || t.xvar < 0 || t.xvar > 3 ||
      (t.xvar == 2 && c->g.nx > 512) || (t.xvar == 3 && c->g.nx > 256) || t.slab < 0 ||
      (t.slab > 0 && 4LL * t.slab > 3LL * c->g.nz) || (t.xyblk && !x_reads_blocked(xa)) ||
      (t.zfuse && !can_fuse(c)))
    return fail(c, FCNS_EINVAL, "a choice this context cannot take");
  if (!zplan.empty()) {
    fcns_status st = set_z_plan(c, zplan);
    if (st) return st;
  }
  c->ygrid = t.ygrid;
  c->ynopf = t.ynopf != 0;
  c->ylines = t.ylines;
  c->ygrid1 = t.ygrid1;
  c->ynopf1 = t.ynopf1 != 0;
  c->ylines1 = t.ylines1;
  c->xvar = t.xvar;
  c->slab = t.slab;
  c->xyblk = t.xyblk;
  c->zfuse = t.zfuse;
  drop_graph(c);
  return FCNS_OK;
}

// Several problems stepped together: step k of every context is enqueued
// before step k + 1 of any, each on its own context stream, so that the
// problems overlap on the device; each context's work is exactly its
// fcns_rk_step.
extern "C" fcns_status fcns_batch_step(fcns_ctx* const* ctxs, int32_t n, const double* dts,
                                       const int32_t* nsteps) {
  if (n < 0 || (n > 0 && (!ctxs || !dts || !nsteps))) return FCNS_EINVAL;
  int most = 0;
  for (int i = 0; i < n; ++i) {
    fcns_ctx* c = ctxs[i];
    if (!c) return FCNS_EINVAL;
    if (!c->has_state) return fail(c, FCNS_ESTATE, "batch_step before set_state");
    if (!(dts[i] > 0.0) || nsteps[i] < 0) return fail(c, FCNS_EINVAL, "need dt > 0, nsteps >= 0");
    most = nsteps[i] > most ? nsteps[i] : most;
  }
  for (int k = 0; k < most; ++k)
    for (int i = 0; i < n; ++i) {
      if (k >= nsteps[i]) continue;
      fcns_ctx* c = ctxs[i];
      const int o = c->prob.rk_order;
      for (int j = 1; j <= o; ++j) {
        if (c->mixed)
          rk_stage<float>(c, j, o, dts[i]);
        else
          rk_stage<double>(c, j, o, dts[i]);
      }
    }
  fcns_status worst = FCNS_OK;
  for (int i = 0; i < n; ++i) {
    if (nsteps[i] > 0 && ctxs[i]->prob.keep_pressure) ctxs[i]->has_pressure = true;
    fcns_status st = finish_steps(ctxs[i], "batch_step");
    if (st == FCNS_ENONFINITE && worst == FCNS_OK) worst = st;
    else if (st != FCNS_OK && st != FCNS_ENONFINITE) return st;
  }
  return worst;
}

// ---------------------------------------------------------------- batch
// Several problems of different shapes stepped together with one launch of
// the fused z pass per RK stage for all of them: each context's x and y
// passes run on its own stream, the batch stream waits for all of them,
// runs the z passes of every problem in one kernel, and every context stream
// waits for that before its next pass.
struct fcns_batch {
  std::vector<fcns_ctx*> ctx;
  int o = 2;
  hipStream_t stream = nullptr;
  hipEvent_t ev_z = nullptr;
  std::vector<hipEvent_t> ev_ctx;
  ZPassDesc* desc = nullptr;      // [o][n] on the device
  std::vector<ZPassDesc> hdesc;   // the host copy they were made from
  std::vector<double> dt;         // per context
  std::vector<double> cj;         // [o][n]
  std::vector<char> fusable;      // per stage: the output buffer is not the input
  long long groups = 0;
  int max_npr = 0;
  bool big = false;
  size_t lds = 0;
};

// The descriptors of every (stage, context) from the contexts as they are
// now (their tables, parameters and buffers), and the launch shape.
static void batch_descriptors(fcns_batch* b, std::vector<ZPassDesc>& h) {
  const int n = (int)b->ctx.size(), o = b->o;
  h.resize((size_t)o * n);
  memset(h.data(), 0, h.size() * sizeof(ZPassDesc));
  b->cj.assign((size_t)o * n, 0.0);
  b->fusable.assign(o, 0);
  b->max_npr = 0;
  b->big = false;
  b->lds = 0;
  for (int j = 1; j <= o; ++j) {
    long long wg = 0;
    for (int i = 0; i < n; ++i) {
      fcns_ctx* c = b->ctx[i];
      cpx<double>* W = (j == 1) ? c->P : c->Q;
      cpx<double>* OUT = (j == o) ? c->P : c->Q;
      b->fusable[j - 1] = OUT != W;
      const double cj = b->dt[i] / (double)(o - j + 1);
      b->cj[(size_t)(j - 1) * n + i] = cj;
      ZPassDesc& d = h[(size_t)(j - 1) * n + i];
      d.a = zargs(c);
      d.a.nonfinite = c->dflag;
      z_part_args<double>(c, W, OUT, cj, c->prob.keep_pressure && j == o, true, d.sa, d.sb);
      d.zb = ZBackArgs{c->MV, c->M};
      d.nf = c->nf;
      d.wg0 = wg;
      wg += z_pass_groups(d.a);
      b->max_npr = std::max(b->max_npr, c->g.npr);
      b->big = b->big || c->big_z;
      b->lds = std::max(b->lds, z_pass_lds(d.a));
    }
    b->groups = wg;
  }
}

static void batch_free(fcns_batch* b) {
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->desc) (void)hipFree(b->desc);
  if (b->ev_z) (void)hipEventDestroy(b->ev_z);
  for (hipEvent_t e : b->ev_ctx)
    if (e) (void)hipEventDestroy(e);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

extern "C" fcns_status fcns_batch_create(fcns_ctx* const* ctxs, int32_t n, const double* dts,
                                         fcns_batch** out) {
  if (!out) return FCNS_EINVAL;
  *out = nullptr;
  if (n < 1 || !ctxs || !dts) return fail(nullptr, FCNS_EINVAL, "need n >= 1 contexts and dts");
  const int o = ctxs[0] ? ctxs[0]->prob.rk_order : 0;
  for (int i = 0; i < n; ++i) {
    fcns_ctx* c = ctxs[i];
    if (!c) return fail(nullptr, FCNS_EINVAL, "NULL context");
    if (!can_fuse(c))
      return fail(c, FCNS_EINVAL, "batched z pass needs FP64 contexts with N' <= 288");
    if (c->prob.rk_order != o) return fail(c, FCNS_EINVAL, "contexts must share rk_order");
    if (!(dts[i] > 0.0)) return fail(c, FCNS_EINVAL, "need dt > 0");
  }
  fcns_batch* b = new fcns_batch();
  b->ctx.assign(ctxs, ctxs + n);
  b->o = o;
  b->dt.assign(dts, dts + n);
  std::vector<ZPassDesc> h;
  batch_descriptors(b, h);
  b->hdesc = h;
  fcns_status st = FCNS_OK;
  if (hipMalloc((void**)&b->desc, h.size() * sizeof(ZPassDesc)) != hipSuccess) {
    batch_free(b);
    return fail(nullptr, FCNS_ENOMEM, "batch descriptors");
  }
  if (hipMemcpy(b->desc, h.data(), h.size() * sizeof(ZPassDesc), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_z, hipEventDisableTiming) != hipSuccess)
    st = FCNS_EDEVICE;
  b->ev_ctx.assign(n, nullptr);
  for (int i = 0; i < n && st == FCNS_OK; ++i)
    if (hipEventCreateWithFlags(&b->ev_ctx[i], hipEventDisableTiming) != hipSuccess)
      st = FCNS_EDEVICE;
  if (st != FCNS_OK) {
    batch_free(b);
    return fail(nullptr, st, "batch set-up");
  }
  *out = b;
  return FCNS_OK;
}

extern "C" fcns_status fcns_batch_run(fcns_batch* b, int32_t nsteps) {
  if (!b) return FCNS_EINVAL;
  if (nsteps < 0) return fail(b->ctx[0], FCNS_EINVAL, "nsteps < 0");
  const int n = (int)b->ctx.size(), o = b->o;
  for (fcns_ctx* c : b->ctx)
    if (!c->has_state) return fail(c, FCNS_ESTATE, "batch_run before set_state");
  // a member retuned (new z tables) or given new parameters since: new
  // descriptors before any launch that reads them
  std::vector<ZPassDesc> h;
  batch_descriptors(b, h);
  if (memcmp(h.data(), b->hdesc.data(), h.size() * sizeof(ZPassDesc)) != 0) {
    fcns_status st = check_hip(b->ctx[0], hipStreamSynchronize(b->stream), "batch_run");
    if (st == FCNS_OK)
      st = check_hip(b->ctx[0], hipMemcpy(b->desc, h.data(), h.size() * sizeof(ZPassDesc),
                                          hipMemcpyHostToDevice), "batch_run");
    if (st != FCNS_OK) return st;
    b->hdesc = h;
  }
  for (int k = 0; k < nsteps; ++k)
    for (int j = 1; j <= o; ++j) {
      for (int i = 0; i < n; ++i) {
        fcns_ctx* c = b->ctx[i];
        nonlinear_from_mixed<double>(c, c->MV, c->nf, true);
        if (b->fusable[j - 1]) {
          (void)hipEventRecord(b->ev_ctx[i], c->stream);
          (void)hipStreamWaitEvent(b->stream, b->ev_ctx[i], 0);
        } else {
          cpx<double>* W = (j == 1) ? c->P : c->Q;
          cpx<double>* OUT = (j == o) ? c->P : c->Q;
          z_part<double>(c, W, OUT, b->cj[(size_t)(j - 1) * n + i],
                         c->prob.keep_pressure && j == o, false);
        }
      }
      if (b->fusable[j - 1]) {
        launch_z_pass_batch(b->desc + (size_t)(j - 1) * n, n, b->groups, b->max_npr, b->big,
                            b->lds, b->stream);
        (void)hipEventRecord(b->ev_z, b->stream);
        for (fcns_ctx* c : b->ctx) (void)hipStreamWaitEvent(c->stream, b->ev_z, 0);
      }
    }
  fcns_status worst = FCNS_OK;
  for (fcns_ctx* c : b->ctx) {
    if (nsteps > 0 && c->prob.keep_pressure) c->has_pressure = true;
    fcns_status st = finish_steps(c, "batch_run");
    if (st == FCNS_ENONFINITE && worst == FCNS_OK) worst = st;
    else if (st != FCNS_OK && st != FCNS_ENONFINITE) return st;
  }
  return worst;
}

extern "C" fcns_status fcns_batch_destroy(fcns_batch* b) {
  if (b) batch_free(b);
  return FCNS_OK;
}

extern "C" fcns_status fcns_get_state(fcns_ctx* c, double* v, double* theta, double* p) {
  if (!c) return FCNS_EINVAL;
  if (!c->has_state) return fail(c, FCNS_ESTATE, "get_state before set_state");
  if (p && !c->has_pressure)
    return fail(c, FCNS_ESTATE, "pressure needs keep_pressure and at least one step");
  const long long M = c->M;
  if (v || theta) {
    // R IFFT of the continued state, then the inverse xy transforms
    launch_z_back<double>(zargs(c), c->big_z, c->P, c->MVT, nullptr, c->S, M, c->nf, c->stream);
    if (v) mixed_to_phys(c, c->MVT, M, 3, v, c->g.nz);
    if (theta && c->nf == 4) mixed_to_phys(c, c->MVT + 3 * M, M, 1, theta, c->g.nz);
  }
  if (p) {
    launch_sub_mean00(c->PM, c->g.npen, c->g.nz, 1.0, c->stream);
    mixed_to_phys(c, c->PM, M, 1, p, c->g.nz);
  }
  return check_launch(c, "get_state");
}

extern "C" fcns_status fcns_rhs_nonlinear(fcns_ctx* c, const double* v, const double* theta,
                                          int32_t filtered, double* nl_v, double* nl_theta) {
  if (!c) return FCNS_EINVAL;
  if (!v || !nl_v) return fail(c, FCNS_EINVAL, "NULL pointer");
  if (theta && c->nf != 4) return fail(c, FCNS_EINVAL, "theta needs a Boussinesq context");
  if (theta && !nl_theta) return fail(c, FCNS_EINVAL, "nl_theta is NULL");
  const int nf = theta ? 4 : 3;
  const long long M = c->M;
  phys_to_mixed(c, v, 3, c->XYB);
  if (theta) phys_to_mixed(c, theta, 1, c->XYB + 3 * M);
  mixed_to_state(c, c->XYB, nf, c->VS, c->MVT);
  nonlinear_from_mixed<double>(c, c->MVT, nf, filtered != 0);
  if (filtered) {
    launch_z_fwd(zargs(c), c->big_z, c->NLB, c->VS, M, c->S, nf, 1, c->stream);
    launch_z_back<double>(zargs(c), c->big_z, c->VS, c->NLB, nullptr, c->S, M, nf, c->stream);
    mixed_to_phys(c, c->NLB, M, 3, nl_v, c->g.nz);
    if (theta) mixed_to_phys(c, c->NLB + 3 * M, M, 1, nl_theta, c->g.nz);
  } else {
    const Geom& g = c->g;
    const long long pfs = (long long)g.nz * g.ny * g.nx;
    launch_x_c2r(xargs(c), c->big_x, c->NLB, nl_v, M, pfs, (long long)g.nz * g.ny, 3, c->stream);
    if (theta)
      launch_x_c2r(xargs(c), c->big_x, c->NLB + 3 * M, nl_theta, M, pfs, (long long)g.nz * g.ny,
                   1, c->stream);
  }
  return check_launch(c, "rhs_nonlinear");
}

extern "C" fcns_status fcns_pressure_project(fcns_ctx* c, const double* v_star, double cj,
                                             double* v_out, double* gradp_wall) {
  if (!c) return FCNS_EINVAL;
  if (!v_star || !v_out) return fail(c, FCNS_EINVAL, "NULL pointer");
  if (!(cj > 0.0)) return fail(c, FCNS_EINVAL, "c must be > 0");
  const long long M = c->M, S = c->S;
  phys_to_mixed(c, v_star, 3, c->XYB);
  launch_z_fwd(zargs(c), c->big_z, c->XYB, c->VS, M, S, 3, 0, c->stream);
  StageBArgs B{};
  for (int i = 0; i < 3; ++i) {
    B.vs[i] = c->VS + i * S;
    B.vout[i] = c->VS + i * S;
  }
  B.gwall = c->GWT;
  B.pmix = nullptr;
  B.c = cj;
  launch_z_stageB(zargs(c), c->big_z, B, c->stream);
  launch_z_back<double>(zargs(c), c->big_z, c->VS, c->MVT, nullptr, S, M, 3, c->stream);
  mixed_to_phys(c, c->MVT, M, 3, v_out, c->g.nz);
  if (gradp_wall) mixed_to_phys(c, c->GWT, 0, 1, gradp_wall, 4);
  return check_launch(c, "pressure_project");
}

// ---------------------------------------------------------------- diagnostics
extern "C" fcns_status fcns_diagnostics(fcns_ctx* c, double* out, int32_t nout) {
  if (!c) return FCNS_EINVAL;
  if (!c->has_state) return fail(c, FCNS_ESTATE, "diagnostics before set_state");
  if (!out || nout < 0) return fail(c, FCNS_EINVAL, "NULL out");
  const Geom& g = c->g;
  const long long M = c->M;
  launch_z_back<double>(zargs(c), c->big_z, c->P, c->MVT, c->MVT + M, c->S, 2 * M, c->nf,
                        c->stream);
  launch_diag_planes(g, c->MVT, M, c->nf, c->DG, c->stream);
  fcns_status st = check_launch(c, "diagnostics");
  if (st != FCNS_OK) return st;
  std::vector<double> pl(5 * (size_t)g.nz);
  cpx<double> corner[4] = {};  // (0,0) mode of du/dz, dtheta/dz at z = 0, Lz
  const long long zt = (long long)(g.nz - 1) * g.npen;
  const cpx<double>* dudz = c->MVT + M;
  const cpx<double>* dtdz = c->MVT + 7 * M;
  if ((st = check_hip(c, hipMemcpyAsync(pl.data(), c->DG, pl.size() * sizeof(double),
                                        hipMemcpyDeviceToHost, c->stream), "diagnostics")) ||
      (st = check_hip(c, hipMemcpyAsync(&corner[0], dudz, sizeof(cpx<double>),
                                        hipMemcpyDeviceToHost, c->stream), "diagnostics")) ||
      (st = check_hip(c, hipMemcpyAsync(&corner[1], dudz + zt, sizeof(cpx<double>),
                                        hipMemcpyDeviceToHost, c->stream), "diagnostics")))
    return st;
  if (c->nf == 4 &&
      ((st = check_hip(c, hipMemcpyAsync(&corner[2], dtdz, sizeof(cpx<double>),
                                         hipMemcpyDeviceToHost, c->stream), "diagnostics")) ||
       (st = check_hip(c, hipMemcpyAsync(&corner[3], dtdz + zt, sizeof(cpx<double>),
                                         hipMemcpyDeviceToHost, c->stream), "diagnostics"))))
    return st;
  if ((st = check_hip(c, hipStreamSynchronize(c->stream), "diagnostics"))) return st;
  const double nxy = (double)g.nx * g.ny, n2 = nxy * nxy;
  double sum[5] = {0, 0, 0, 0, 0};
  for (int z = 0; z < g.nz; ++z)
    for (int q = 0; q < 5; ++q) sum[q] += pl[5 * z + q];
  const double* b = &pl[0];
  const double* t = &pl[5 * (size_t)(g.nz - 1)];
  const double nu = c->prob.nu, delta = 0.5 * g.lz;
  const double dub = corner[0].x / nxy, dut = corner[1].x / nxy;
  double v[FCNS_NDIAG];
  v[0] = 0.5 * (sum[0] + sum[1] + sum[2]) / n2 / g.nz;     // kinetic energy
  v[1] = sum[4] / n2 / g.nz;                                // <(div v)^2>
  v[2] = (b[0] + b[1]) / n2;                                // slip, bottom
  v[3] = (t[0] + t[1]) / n2;                                // slip, top
  v[4] = b[2] / n2;                                         // <w^2>, bottom
  v[5] = t[2] / n2;                                         // <w^2>, top
  v[6] = dub;                                               // <du/dz>, bottom
  v[7] = dut;                                               // <du/dz>, top
  v[8] = nu > 0 ? sqrt(nu * fabs(dub)) * delta / nu : 0.0;  // Re_tau, bottom
  v[9] = nu > 0 ? sqrt(nu * fabs(dut)) * delta / nu : 0.0;  // Re_tau, top
  if (c->nf == 4) {
    v[10] = 1.0 - corner[2].x / nxy / c->prob.gamma;        // Nu, bottom
    v[11] = 1.0 - corner[3].x / nxy / c->prob.gamma;        // Nu, top
    v[12] = sum[3] / n2 / g.nz;                              // <theta^2>
  } else {
    v[10] = v[11] = NAN;
    v[12] = 0.0;
  }
  for (int i = 0; i < nout && i < FCNS_NDIAG; ++i) out[i] = v[i];
  return FCNS_OK;
}

extern "C" fcns_status fcns_spectra(fcns_ctx* c, int32_t field, int32_t z, double* ex,
                                    double* ey) {
  if (!c) return FCNS_EINVAL;
  if (!c->has_state) return fail(c, FCNS_ESTATE, "spectra before set_state");
  if (field < 0 || field >= c->nf || z < 0 || z >= c->g.nz || !ex || !ey)
    return fail(c, FCNS_EINVAL, "bad field, height or NULL");
  const Geom& g = c->g;
  launch_z_back<double>(zargs(c), c->big_z, c->P + field * c->S, c->MVT, nullptr, c->S, c->M, 1,
                        c->stream);
  double* dex = c->DG + 5 * (size_t)g.nz;
  double* dey = dex + g.nkx;
  launch_spectra(g, c->MVT, z, dex, dey, c->stream);
  fcns_status st = check_launch(c, "spectra");
  if (st) return st;
  if ((st = check_hip(c, hipMemcpyAsync(ex, dex, g.nkx * sizeof(double), hipMemcpyDeviceToHost,
                                        c->stream), "spectra")) ||
      (st = check_hip(c, hipMemcpyAsync(ey, dey, g.ny * sizeof(double), hipMemcpyDeviceToHost,
                                        c->stream), "spectra")))
    return st;
  return check_hip(c, hipStreamSynchronize(c->stream), "spectra");
}

extern "C" fcns_status fcns_get_spectral(fcns_ctx* c, int32_t field, double* out) {
  if (!c) return FCNS_EINVAL;
  if (!c->has_state) return fail(c, FCNS_ESTATE, "no state");
  if (field < 0 || field >= c->nf || !out) return fail(c, FCNS_EINVAL, "bad field or NULL");
  const size_t w = c->g.nkx * sizeof(cpx<double>), ld = c->g.nkxp * sizeof(cpx<double>);
  return check_hip(c,
                   hipMemcpy2DAsync(out, w, c->P + field * c->S, ld, w,
                                    (size_t)c->g.npr * c->g.ny, hipMemcpyDeviceToDevice,
                                    c->stream),
                   "get_spectral");
}

extern "C" fcns_status fcns_set_spectral(fcns_ctx* c, const double* const* fields,
                                         const double* wall_grad) {
  if (!c) return FCNS_EINVAL;
  if (!fields) return fail(c, FCNS_EINVAL, "NULL fields");
  for (int f = 0; f < c->nf; ++f) {
    if (!fields[f]) return fail(c, FCNS_EINVAL, "NULL field");
    const size_t w = c->g.nkx * sizeof(cpx<double>), ld = c->g.nkxp * sizeof(cpx<double>);
    fcns_status st = check_hip(c,
                               hipMemcpy2DAsync(c->P + f * c->S, ld, fields[f], w, w,
                                                (size_t)c->g.npr * c->g.ny,
                                                hipMemcpyDeviceToDevice, c->stream),
                               "set_spectral");
    if (st != FCNS_OK) return st;
  }
  if (wall_grad) {
    const size_t w = c->g.nkx * sizeof(cpx<double>), ld = c->g.nkxp * sizeof(cpx<double>);
    fcns_status st = check_hip(c,
                               hipMemcpy2DAsync(c->GW, ld, wall_grad, w, w, (size_t)4 * c->g.ny,
                                                hipMemcpyDeviceToDevice, c->stream),
                               "set_spectral");
    if (st != FCNS_OK) return st;
  } else {
    launch_fill(c->GW, 4 * c->g.npen, c->stream);
  }
  state_to_mv(c, c->P);
  clear_flag(c);
  fcns_status st = check_launch(c, "set_spectral");
  if (st == FCNS_OK) {
    c->has_state = true;
    c->has_pressure = false;
  }
  return st;
}

extern "C" fcns_status fcns_get_wall_grad(fcns_ctx* c, double* out) {
  if (!c || !out) return FCNS_EINVAL;
  const size_t w = c->g.nkx * sizeof(cpx<double>), ld = c->g.nkxp * sizeof(cpx<double>);
  return check_hip(c,
                   hipMemcpy2DAsync(out, w, c->GW, ld, w, (size_t)4 * c->g.ny,
                                    hipMemcpyDeviceToDevice, c->stream),
                   "get_wall_grad");
}

// ---------------------------------------------------------------- timing
extern "C" fcns_status fcns_set_timing_mask(fcns_ctx* c, int32_t mask) {
  if (!c) return FCNS_EINVAL;
  if (mask & ~((1 << T_NCLS) - 1)) return fail(c, FCNS_EINVAL, "timing mask names no class");
  if (mask && c->evpool.empty()) {
    c->evpool.resize(4096);
    for (auto& e : c->evpool)
      if (hipEventCreate(&e) != hipSuccess) return fail(c, FCNS_EDEVICE, "hipEventCreate failed");
  }
  timing_flush(c);
  c->timing = mask != 0;
  c->tmask = (uint32_t)mask;
  return FCNS_OK;
}

extern "C" fcns_status fcns_set_timing(fcns_ctx* c, int32_t enable) {
  return fcns_set_timing_mask(c, enable ? (1 << T_NCLS) - 1 : 0);
}

extern "C" fcns_status fcns_timing_reset(fcns_ctx* c) {
  if (!c) return FCNS_EINVAL;
  timing_flush(c);
  for (int i = 0; i < T_NCLS; ++i) {
    c->tms[i] = 0.0;
    c->tcnt[i] = 0;
  }
  return FCNS_OK;
}

extern "C" fcns_status fcns_timing_report(fcns_ctx* c, int32_t max, int32_t* n, char* names,
                                          int64_t* counts, double* ms) {
  if (!c || !n) return FCNS_EINVAL;
  timing_flush(c);
  const int k = max < T_NCLS ? max : T_NCLS;
  for (int i = 0; i < k; ++i) {
    if (names) {
      strncpy(names + 32 * i, kTimingNames[i], 31);
      names[32 * i + 31] = 0;
    }
    if (counts) counts[i] = c->tcnt[i];
    if (ms) ms[i] = c->tms[i];
  }
  *n = k;
  return FCNS_OK;
}
