// Shared device/host helpers for the FC-Gram pseudospectral step on gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcns {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
// Streaming accesses (data a workgroup loads or stores once): the
// nontemporal hint keeps those lines from displacing the ones it reuses.
template <typename T>
__device__ __forceinline__ cpx<T> ld_stream(const cpx<T>* p) {
  using V = T __attribute__((ext_vector_type(2)));
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return mk(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void st_stream(cpx<T>* p, cpx<T> a) {
  using V = T __attribute__((ext_vector_type(2)));
  const V v = {a.x, a.y};
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return mk(a.x + b.x, a.y + b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return mk(a.x - b.x, a.y - b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, T s) {
  return mk(a.x * s, a.y * s);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) {
  return mk(a.x, -a.y);
}
// i * a
template <typename T>
__host__ __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
  return mk(-a.y, a.x);
}
// -i * a
template <typename T>
__host__ __device__ __forceinline__ cpx<T> mul_mi(cpx<T> a) {
  return mk(a.y, -a.x);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> zero() {
  return mk(T(0), T(0));
}

// Convert between precisions (FP64 state, FP32 transforms in mixed mode).
template <typename D, typename S>
__host__ __device__ __forceinline__ cpx<D> cvt(cpx<S> a) {
  return mk(static_cast<D>(a.x), static_cast<D>(a.y));
}

// Geometry of one problem, passed by value to every kernel.
struct Geom {
  int nx, ny, nz;       // physical grid; nz includes both walls
  int nkx;              // nx/2 + 1 stored kx modes
  int nkxp;             // row stride in kx: nkx rounded up to a multiple of 4 (64 B)
  int npr;              // N' = nz + C, continued points in z
  int C, d;             // FC continuation / matching points
  long long npen;       // pencil slots = nkxp * ny (kx >= nkx are padding)
  double lx, ly, lz;    // box
  double dz, lzp;       // dz = lz/(nz-1), Lz' = N' dz
  double kxs, kys, kzs; // 2 pi / lx, 2 pi / ly, 2 pi / Lz'
};

// Wavenumber of FFT index i (true value; the Nyquist index of an even n maps
// to -n/2 as in numpy's fftfreq) and its odd-derivative version (Nyquist 0).
__host__ __device__ __forceinline__ double k_true(int i, int n, double scale) {
  int m = (2 * i < n) ? i : i - n;
  return scale * (double)m;
}
__host__ __device__ __forceinline__ double k_odd(int i, int n, double scale) {
  if (2 * i == n) return 0.0;
  int m = (2 * i < n) ? i : i - n;
  return scale * (double)m;
}

}  // namespace fcns
