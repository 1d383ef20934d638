// Vector kernels of the Krylov, Chebyshev and coarse-grid drivers.
//
// Inner products are 2-norm products over unique free nodes, computed on
// E-vectors with the weight w = mask / multiplicity.  Every reduction uses a
// fixed launch shape and a fixed summation tree (per-thread strided partial
// sums, an LDS tree per block, then the block partials summed in block
// order), so results are bitwise repeatable.  The outer Krylov reductions
// sum the block partials in a second, one-workgroup launch (k_finish); the
// E-vector coarse CG (a coarsest level other than the assembled p = 1 one)
// keeps the single-launch form, where the last block to finish, found with a
// ticket counter, sums them (last_block_sum).
#include <algorithm>
#include <initializer_list>
#include <type_traits>

#include "sem_internal.h"

namespace sem {

static inline unsigned nb(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }
static inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Streams read or written once per pass may go non-temporal (NT): they then
// do not displace the lines that a kernel's neighbour reads hit in L2 (the
// deferred-step forms below: 1-2 ms per solve on the 32^3, p = 7 benchmark).
template <bool NT, typename T>
__device__ inline T ldn(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ inline void stn(T *p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// 16-byte vectors (4 floats or 2 doubles) for the pointwise kernels: one load
// or store instruction per operand and thread; arithmetic acts per element
template <typename T>
struct V16;
template <>
struct V16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct V16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
// the vector form applies when n is a multiple of the width and every
// operand is 16-byte aligned
template <typename T>
static inline bool vec16_ok(int64_t n, std::initializer_list<const void *> ps) {
  if (n % (int64_t)(16 / sizeof(T)) != 0) return false;
  for (const void *q : ps)
    if (q && !aligned16(q)) return false;
  return true;
}
static inline unsigned red_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > kRedBlocks) g = kRedBlocks;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// elementwise
template <typename T>
__global__ void k_scale(int64_t n, const T *__restrict__ w, const T *__restrict__ x,
                        T *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[t] = w[t] * x[t];
}
template <typename T>
void launch_scale(int64_t n, const T *w, const T *x, T *y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale<T>, dim3(nb(n, 256)), dim3(256), 0, s, n, w, x, y);
  SEM_LAUNCH("k_scale");
}
template void launch_scale<double>(int64_t, const double *, const double *, double *, hipStream_t);
template void launch_scale<float>(int64_t, const float *, const float *, float *, hipStream_t);

__global__ void k_d2f(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[t] = (float)x[t];
}
__global__ void k_f2d(int64_t n, const float *__restrict__ x, double *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[t] = (double)x[t];
}
void launch_copy_cvt_d2f(int64_t n, const double *x, float *y, hipStream_t s) {
  hipLaunchKernelGGL(k_d2f, dim3(nb(n, 256)), dim3(256), 0, s, n, x, y);
  SEM_LAUNCH("k_d2f");
}
void launch_copy_cvt_f2d(int64_t n, const float *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_f2d, dim3(nb(n, 256)), dim3(256), 0, s, n, x, y);
  SEM_LAUNCH("k_f2d");
}

template <typename T>
__global__ void k_axpby(int64_t n, T a, const T *__restrict__ x, T b, T *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  // b = 0 overwrites y without reading it (y may be uninitialised: 0 * NaN = NaN)
  y[t] = b == T(0) ? a * x[t] : a * x[t] + b * y[t];
}
template <typename T>
void launch_axpby(int64_t n, T a, const T *x, T b, T *y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby<T>, dim3(nb(n, 256)), dim3(256), 0, s, n, a, x, b, y);
  SEM_LAUNCH("k_axpby");
}
template void launch_axpby<double>(int64_t, double, const double *, double, double *, hipStream_t);
template void launch_axpby<float>(int64_t, float, const float *, float, float *, hipStream_t);

template <typename T>
__global__ void k_sub(int64_t n, const T *__restrict__ a, const T *__restrict__ b,
                      T *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[t] = a[t] - b[t];
}
template <typename T>
void launch_sub(int64_t n, const T *a, const T *b, T *y, hipStream_t s) {
  hipLaunchKernelGGL(k_sub<T>, dim3(nb(n, 256)), dim3(256), 0, s, n, a, b, y);
  SEM_LAUNCH("k_sub");
}
template void launch_sub<double>(int64_t, const double *, const double *, double *, hipStream_t);
template void launch_sub<float>(int64_t, const float *, const float *, float *, hipStream_t);

// one pass of the loop body: x += d_k; r -= S A d_k (= t); d = a d_k + c r
// (xz: x is zero on entry and is not read)
// t read as assembled (XD::value false), or with the deferred x step of the
// gather-scatter taken on the way (16-byte vectors VT of T; a vector never
// straddles an element row, so only its first lane can be an i = 0 node and
// only its last an i = p node).  The kernels that read this way take their
// blocks in XCD-contiguous order (xcd_block), so the x-neighbour copies they
// read mostly come from rows the same XCD reads: its own L2.
struct XDev {
  unsigned nex, ney, N, p, vrow, vel, vside;  // vectors per row, per element, per right side
  int bc0, bc1, bc2, bc3;
  int y;  // the y step is deferred too (taken before the x step)
};
template <typename XD, typename VT>
__device__ inline VT read_t(const VT *__restrict__ tv, int64_t m, const XDev &f) {
  VT v = tv[m];
  if constexpr (XD::value) {
    using T = std::decay_t<decltype(v[0])>;
    constexpr int W = sizeof(VT) / sizeof(T);
    const T *__restrict__ ts = reinterpret_cast<const T *>(tv);
    const unsigned mq = (unsigned)(m % f.vside);
    const unsigned e = mq / f.vel;
    const unsigned vi = mq - e * f.vel;
    const unsigned i0 = vi % f.vrow * W;
    const unsigned ex = e % f.nex;
    const int64_t q = m * W;
    const int64_t N3 = (int64_t)f.vel * W;
    // y step (rows j = 0 and j = p): (p-row of the lower element + 0-row of the
    // upper), Dirichlet y-faces zero; ys gives the same for one x-neighbour value
    int ymode = 0;  // 0 none, 1 j = 0 with a lower copy, 2 j = p with an upper copy, 3 zero
    int64_t yoff = 0;
    if (f.y) {
      const unsigned j = (vi / f.vrow) % f.N;
      const unsigned ey = (e / f.nex) % f.ney;
      yoff = (int64_t)f.nex * N3 - (int64_t)f.p * f.N;
      if (j == 0)
        ymode = ey > 0 ? 1 : (f.bc2 ? 3 : 0);
      else if (j == f.p)
        ymode = ey + 1 < f.ney ? 2 : (f.bc3 ? 3 : 0);
      if (ymode == 1)
        v = tv[m - yoff / W] + v;
      else if (ymode == 2)
        v = v + tv[m + yoff / W];
      else if (ymode == 3)
        v = VT(T(0));
    }
    auto ys = [&](int64_t idx) -> T {
      const T own = ts[idx];
      if (ymode == 1) return ts[idx - yoff] + own;
      if (ymode == 2) return own + ts[idx + yoff];
      if (ymode == 3) return T(0);
      return own;
    };
    if (i0 == 0) {
      if (ex > 0)
        v[0] = ys(q - N3 + f.p) + v[0];
      else if (f.bc0)
        v[0] = T(0);
    }
    if (i0 + W - 1 == f.p) {
      if (ex + 1 < f.nex)
        v[W - 1] = v[W - 1] + ys(q + (W - 1) - f.p + N3);
      else if (f.bc1)
        v[W - 1] = T(0);
    }
  }
  return v;
}

template <typename T, typename XD = std::false_type>
__global__ void k_cheb_update(int64_t n, T *__restrict__ x, T *__restrict__ r, T *__restrict__ d,
                              const T *__restrict__ tv, T a, T c, int xz, XDev f) {
  int64_t t = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  T dk = d[t];
  x[t] = xz ? dk : x[t] + dk;
  T rn = r[t] - read_t<XD>(tv, t, f);
  r[t] = rn;
  d[t] = a * dk + c * rn;
}
template <typename T>
bool cheb_can_defer_x(int N, int64_t n, std::initializer_list<const void *> ps) {
  return N % (int)(16 / sizeof(T)) == 0 && vec16_ok<T>(n, ps);
}
template bool cheb_can_defer_x<float>(int, int64_t, std::initializer_list<const void *>);
template bool cheb_can_defer_x<double>(int, int64_t, std::initializer_list<const void *>);

template <typename T>
static XDev xdev(const XDefer &xd) {
  constexpr unsigned W = 16 / sizeof(T);
  XDev f{};
  if (!xd.on) return f;
  if (xd.N % (int)W != 0 || xd.nloc % ((int64_t)xd.N * xd.N * xd.N) != 0)
    fail(SEM_EINVAL, "deferred x step: vectors straddle element rows");
  f.nex = (unsigned)xd.nex;
  f.N = (unsigned)xd.N;
  f.p = (unsigned)xd.N - 1;
  f.vrow = (unsigned)xd.N / W;
  f.vel = (unsigned)(xd.N * xd.N * xd.N) / W;
  f.vside = (unsigned)(xd.nloc / W);
  f.bc0 = xd.bc0;
  f.bc1 = xd.bc1;
  f.y = xd.y ? 1 : 0;
  f.ney = (unsigned)xd.ney;
  f.bc2 = xd.bc2;
  f.bc3 = xd.bc3;
  return f;
}

template <typename T>
void launch_cheb_update(int64_t n, T *x, T *r, T *d, const T *t, T a, T c, hipStream_t s,
                        bool x_zero, const XDefer &xd) {
  const XDev f = xdev<T>(xd);
  if (vec16_ok<T>(n, {x, r, d, t})) {
    using VT = typename V16<T>::type;
    const int64_t m = n / (int64_t)(16 / sizeof(T));
    if (xd.on)
      hipLaunchKernelGGL((k_cheb_update<VT, std::true_type>), dim3(nb(m, 256)), dim3(256), 0, s, m,
                         (VT *)x, (VT *)r, (VT *)d, (const VT *)t, (VT)a, (VT)c, (int)x_zero, f);
    else
      hipLaunchKernelGGL((k_cheb_update<VT>), dim3(nb(m, 256)), dim3(256), 0, s, m, (VT *)x,
                         (VT *)r, (VT *)d, (const VT *)t, (VT)a, (VT)c, (int)x_zero, f);
  } else {
    if (xd.on) fail(SEM_EINVAL, "deferred x step needs the vector form");
    hipLaunchKernelGGL((k_cheb_update<T>), dim3(nb(n, 256)), dim3(256), 0, s, n, x, r, d, t, a, c,
                       (int)x_zero, f);
  }
  SEM_LAUNCH("k_cheb_update");
}
template void launch_cheb_update<double>(int64_t, double *, double *, double *, const double *,
                                         double, double, hipStream_t, bool, const XDefer &);
template void launch_cheb_update<float>(int64_t, float *, float *, float *, const float *, float,
                                        float, hipStream_t, bool, const XDefer &);

// The first pass of the loop without forming d_0 = r_0 / theta beforehand: A
// and S are linear, so the caller applies them to r_0 and this pass scales
// (tv = S A r_0).  x += d_0; r -= tv / theta; d = a d_0 + c r; with `last` the
// closing x += d as well (r and d then unwritten).  xz: x is zero on entry.
template <typename T, typename XD = std::false_type, bool NTL = false>
__global__ void k_cheb_first(int64_t n, T *__restrict__ x, T *__restrict__ r, T *__restrict__ d,
                             const T *__restrict__ tv, T inv_theta, T a, T c, int xz, int last,
                             XDev f) {
  int64_t t = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const T r0 = ldn<NTL>(r + t);
  const T d0 = r0 * inv_theta;
  const T x1 = xz ? d0 : ldn<NTL>(x + t) + d0;
  const T rn = r0 - read_t<XD>(tv, t, f) * inv_theta;
  const T dn = a * d0 + c * rn;
  if (last) {
    x[t] = dn + x1;
  } else {
    x[t] = x1;
    r[t] = rn;
    d[t] = dn;
  }
}
template <typename T>
void launch_cheb_first(int64_t n, T *x, T *r, T *d, const T *t, T inv_theta, T a, T c,
                       bool x_zero, bool last, hipStream_t s, const XDefer &xd) {
  const XDev f = xdev<T>(xd);
  if (vec16_ok<T>(n, {x, r, d, t})) {
    using VT = typename V16<T>::type;
    const int64_t m = n / (int64_t)(16 / sizeof(T));
    if (xd.on)  // r and x streamed non-temporally
      hipLaunchKernelGGL((k_cheb_first<VT, std::true_type, true>), dim3(nb(m, 256)), dim3(256), 0,
                         s, m, (VT *)x, (VT *)r, (VT *)d, (const VT *)t, (VT)inv_theta, (VT)a,
                         (VT)c, (int)x_zero, (int)last, f);
    else
      hipLaunchKernelGGL((k_cheb_first<VT>), dim3(nb(m, 256)), dim3(256), 0, s, m, (VT *)x,
                         (VT *)r, (VT *)d, (const VT *)t, (VT)inv_theta, (VT)a, (VT)c,
                         (int)x_zero, (int)last, f);
  } else {
    if (xd.on) fail(SEM_EINVAL, "deferred x step needs the vector form");
    hipLaunchKernelGGL((k_cheb_first<T>), dim3(nb(n, 256)), dim3(256), 0, s, n, x, r, d, t,
                       inv_theta, a, c, (int)x_zero, (int)last, f);
  }
  SEM_LAUNCH("k_cheb_first");
}
template void launch_cheb_first<double>(int64_t, double *, double *, double *, const double *,
                                        double, double, double, bool, bool, hipStream_t,
                                        const XDefer &);
template void launch_cheb_first<float>(int64_t, float *, float *, float *, const float *, float,
                                       float, float, bool, bool, hipStream_t, const XDefer &);

// the last pass of the loop and the closing x += d in one: r and d are not
// needed afterwards, so only x is written (same roundings as the two passes)
template <typename T, typename XD = std::false_type, bool NTL = false, bool NTS = false>
__global__ void k_cheb_last(int64_t n, T *__restrict__ x, const T *__restrict__ r,
                            const T *__restrict__ d, const T *__restrict__ tv, T a, T c, int xz,
                            XDev f) {
  int64_t t = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const T dk = ldn<NTL>(d + t);
  const T x1 = xz ? dk : ldn<NTL>(x + t) + dk;
  const T rn = ldn<NTL>(r + t) - read_t<XD>(tv, t, f);
  const T dn = a * dk + c * rn;
  stn<NTS>(x + t, dn + x1);
}
template <typename T>
void launch_cheb_last(int64_t n, T *x, const T *r, const T *d, const T *t, T a, T c, hipStream_t s,
                      bool x_zero, const XDefer &xd) {
  const XDev f = xdev<T>(xd);
  if (vec16_ok<T>(n, {x, r, d, t})) {
    using VT = typename V16<T>::type;
    const int64_t m = n / (int64_t)(16 / sizeof(T));
    if (xd.on)  // d, x, r and the new x streamed non-temporally
      hipLaunchKernelGGL((k_cheb_last<VT, std::true_type, true, true>), dim3(nb(m, 256)),
                         dim3(256), 0, s, m, (VT *)x, (const VT *)r, (const VT *)d, (const VT *)t,
                         (VT)a, (VT)c, (int)x_zero, f);
    else
      hipLaunchKernelGGL((k_cheb_last<VT>), dim3(nb(m, 256)), dim3(256), 0, s, m, (VT *)x,
                         (const VT *)r, (const VT *)d, (const VT *)t, (VT)a, (VT)c, (int)x_zero,
                         f);
  } else {
    if (xd.on) fail(SEM_EINVAL, "deferred x step needs the vector form");
    hipLaunchKernelGGL((k_cheb_last<T>), dim3(nb(n, 256)), dim3(256), 0, s, n, x, r, d, t, a, c,
                       (int)x_zero, f);
  }
  SEM_LAUNCH("k_cheb_last");
}
template void launch_cheb_last<double>(int64_t, double *, const double *, const double *,
                                       const double *, double, double, hipStream_t, bool,
                                       const XDefer &);
template void launch_cheb_last<float>(int64_t, float *, const float *, const float *,
                                      const float *, float, float, hipStream_t, bool,
                                      const XDefer &);

__global__ void k_jacobi_inv(int64_t n, const double *__restrict__ diag, const double *__restrict__ w,
                             double *__restrict__ dinv, float *__restrict__ dinv32) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double v = (w[t] != 0.0) ? 1.0 / diag[t] : 0.0;
  dinv[t] = v;
  if (dinv32) dinv32[t] = (float)v;
}
void launch_jacobi_inv(int64_t n, const double *diag, const double *w, double *dinv, float *dinv32,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_jacobi_inv, dim3(nb(n, 256)), dim3(256), 0, s, n, diag, w, dinv, dinv32);
  SEM_LAUNCH("k_jacobi_inv");
}

template <typename T>
__global__ void k_copy(int64_t n, const T *__restrict__ x, T *__restrict__ y) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) y[t] = x[t];
}
template <typename T>
void launch_copy(int64_t n, const T *x, T *y, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<T>, dim3(nb(n, 256)), dim3(256), 0, s, n, x, y);
  SEM_LAUNCH("k_copy");
}
template void launch_copy<double>(int64_t, const double *, double *, hipStream_t);
template void launch_copy<float>(int64_t, const float *, float *, hipStream_t);

__global__ void k_fill(int64_t n, double v, double *x) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}
__global__ void k_fillf(int64_t n, float v, float *x) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}
void launch_fill(int64_t n, double v, double *x, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(nb(n, 256)), dim3(256), 0, s, n, v, x);
  SEM_LAUNCH("k_fill");
}
void launch_fillf(int64_t n, float v, float *x, hipStream_t s) {
  hipLaunchKernelGGL(k_fillf, dim3(nb(n, 256)), dim3(256), 0, s, n, v, x);
  SEM_LAUNCH("k_fillf");
}

// ---------------------------------------------------------------------------
// reductions
template <int ND>
__device__ inline void block_reduce(double (&acc)[ND], double (*sh)[256]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < ND; ++j) sh[j][tid] = acc[j];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int j = 0; j < ND; ++j) sh[j][tid] += sh[j][tid + h];
    }
    __syncthreads();
  }
}

// Writes this block's partials; returns true in the block that finishes last,
// after the block partials have been summed in block order into acc (thread 0).
template <int ND>
__device__ inline bool last_block_sum(double (&acc)[ND], double *partials, unsigned *counter) {
  __shared__ double sh[ND][256];
  __shared__ bool is_last;
  block_reduce<ND>(acc, sh);
  const int tid = threadIdx.x;
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) partials[blockIdx.x * 8 + j] = sh[j][0];
    __threadfence();
    unsigned ticket = atomicAdd(counter, 1u);
    is_last = (ticket == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  for (int b = tid; b < (int)gridDim.x; b += 256) {
#pragma unroll
    for (int j = 0; j < ND; ++j)
      acc[j] += __hip_atomic_load(&partials[b * 8 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_reduce<ND>(acc, sh);
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = sh[j][0];
  if (tid == 0) *counter = 0u;
  return true;
}

// The hot reductions end in two launches instead: each block writes its
// partials, and a one-workgroup kernel sums them in the same order as the
// last-block path (so the results are the same).  A ticket counter taken by
// every block serialises on one address (about 45 ns a block), which at 1024
// blocks costs more than the second launch.
template <int ND>
__device__ inline void block_partials(double (&acc)[ND], double *partials, int stride = 8) {
  __shared__ double sh[ND][256];
  block_reduce<ND>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) partials[blockIdx.x * stride + j] = sh[j][0];
  }
}
// block b's partials at partials[b * stride + j], nd <= stride <= 8, within
// the buffer's 8 kRedBlocks doubles: stride 8 for up to eight sums over
// kRedBlocks blocks, or densely packed (stride nd) over more blocks
template <int ND>
__global__ __launch_bounds__(256) void k_finish(int nb, const double *__restrict__ partials,
                                                double *out, int stride) {
  __shared__ double sh[ND][256];
  double acc[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
#pragma unroll
    for (int j = 0; j < ND; ++j) acc[j] += partials[b * stride + j];
  }
  block_reduce<ND>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < ND; ++j) out[j] = sh[j][0];
  }
}
static void launch_finish(int nd, unsigned nblocks, const double *partials, double *out,
                          hipStream_t s, int stride = 8) {
  if (stride < nd || stride > 8 || (uint64_t)nblocks * stride > 8u * kRedBlocks)
    fail(SEM_EINVAL, "reduction partials: more than the buffer holds");
  switch (nd) {
    case 1: hipLaunchKernelGGL(k_finish<1>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
    case 2: hipLaunchKernelGGL(k_finish<2>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
    case 3: hipLaunchKernelGGL(k_finish<3>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
    case 4: hipLaunchKernelGGL(k_finish<4>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
    case 5: hipLaunchKernelGGL(k_finish<5>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
    case 6: hipLaunchKernelGGL(k_finish<6>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
    case 7: hipLaunchKernelGGL(k_finish<7>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
    default: hipLaunchKernelGGL(k_finish<8>, dim3(1), dim3(256), 0, s, (int)nblocks, partials, out, stride); break;
  }
  SEM_LAUNCH("k_finish");
}

struct Ptr4 {
  const double *p[4];
};

// out = sum of n partial values in a fixed order: one workgroup of 1024
// threads, eight loads in flight per thread and step (into four running sums),
// then an LDS tree
__global__ __launch_bounds__(1024) void k_sum_partials(int64_t n, const double *__restrict__ part,
                                                       double *out) {
  __shared__ double sh[1024];
  const int tid = threadIdx.x;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = 0; i0 < n; i0 += 8 * 1024) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + u * 1024 + tid;
      v[u] = i < n ? part[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u & 3] += v[u];
  }
  sh[tid] = (a[0] + a[1]) + (a[2] + a[3]);
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (tid < h) sh[tid] += sh[tid + h];
    __syncthreads();
  }
  if (tid == 0) out[0] = sh[0];
}
void launch_sum_partials(int64_t n, const double *part, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, n, part, out);
  SEM_LAUNCH("k_sum_partials");
}

// per-thread strided pairs (16-byte loads when every operand is 16-byte
// aligned), two partial sums per product; an odd last entry goes to the
// first thread
template <typename V>
__device__ inline double2 ld2(const double *p, int64_t t) {
  if constexpr (V::value) return reinterpret_cast<const double2 *>(p)[t];
  return make_double2(p[2 * t], p[2 * t + 1]);
}
// the dot weights mask/multiplicity (0, 1, 1/2, 1/4, 1/8) are exact in FP32:
// the FP32 copy gives the same products with half the weight traffic
template <typename V>
__device__ inline double2 ld2(const float *p, int64_t t) {
  if constexpr (V::value) {
    const float2 v = reinterpret_cast<const float2 *>(p)[t];
    return make_double2((double)v.x, (double)v.y);
  }
  return make_double2((double)p[2 * t], (double)p[2 * t + 1]);
}
template <int ND, typename V, typename WT>
__global__ __launch_bounds__(256) void k_wdots(int64_t n, const WT *__restrict__ w, Ptr4 a,
                                               Ptr4 b, double *partials) {
  double acc[ND], acc2[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = acc2[j] = 0.0;
  const int64_t n2 = n / 2;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t t = t0; t < n2; t += (int64_t)gridDim.x * blockDim.x) {
    const double2 wt = ld2<V>(w, t);
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      const double2 x = ld2<V>(a.p[j], t);
      const double2 y = ld2<V>(b.p[j], t);
      acc[j] += wt.x * x.x * y.x;
      acc2[j] += wt.y * x.y * y.y;
    }
  }
  if (t0 == 0 && (n & 1)) {
#pragma unroll
    for (int j = 0; j < ND; ++j) acc[j] += (double)w[n - 1] * a.p[j][n - 1] * b.p[j][n - 1];
  }
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] += acc2[j];
  block_partials<ND>(acc, partials);
}

// FCG step: x += alpha p, r -= alpha q, and (r, r)_w of the new r, with
// alpha = (r, z) / (p, q) formed from the device scalars (0 when (p, q) <= 0:
// the breakdown leaves x and r as they are; the host reads (p, q) afterwards)
template <typename V>
__device__ inline void st2(double *p, int64_t t, double2 v) {
  if constexpr (V::value) {
    reinterpret_cast<double2 *>(p)[t] = v;
  } else {
    p[2 * t] = v.x;
    p[2 * t + 1] = v.y;
  }
}
// XD: q arrives without the x and y steps of its gather-scatter, which are
// taken as it is read (the Chebyshev updates' read_t)
// NT-capable reads of the 16-byte vector form
template <bool NT>
__device__ inline double2 ld2n(const double *p, int64_t t) {
  using VT = V16<double>::type;
  const VT v = ldn<NT>(reinterpret_cast<const VT *>(p) + t);
  return make_double2(v[0], v[1]);
}
template <bool NT>
__device__ inline double2 ld2n(const float *p, int64_t t) {
  typedef float F2 __attribute__((ext_vector_type(2)));
  const F2 v = ldn<NT>(reinterpret_cast<const F2 *>(p) + t);
  return make_double2((double)v[0], (double)v[1]);
}
template <typename V, typename WT, typename XD = std::false_type, bool NTL = false>
__global__ __launch_bounds__(256) void k_fcg_xr(int64_t n, const double *__restrict__ rz,
                                                const double *__restrict__ pq,
                                                const WT *__restrict__ w,
                                                const double *__restrict__ p,
                                                const double *__restrict__ q, double *__restrict__ x,
                                                double *__restrict__ r, float *__restrict__ rf,
                                                double *partials, int pstride, XDev f) {
  const double pqv = *pq;
  const double alpha = pqv > 0.0 ? *rz / pqv : 0.0;
  double acc[1] = {0.0}, acc2 = 0.0;
  const int64_t n2 = n / 2;
  const int64_t t0 = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t t = t0; t < n2; t += (int64_t)gridDim.x * blockDim.x) {
    double2 qv;
    if constexpr (XD::value) {
      using VT = typename V16<double>::type;
      const VT qq = read_t<XD>(reinterpret_cast<const VT *>(q), t, f);
      qv = make_double2(qq[0], qq[1]);
    } else {
      qv = ld2<V>(q, t);
    }
    double2 pv, wt, xv, rv;
    if constexpr (NTL) {
      static_assert(V::value, "non-temporal reads take the vector form");
      pv = ld2n<true>(p, t);
      wt = ld2n<true>(w, t);
      xv = ld2n<true>(x, t);
      rv = ld2n<true>(r, t);
    } else {
      pv = ld2<V>(p, t);
      wt = ld2<V>(w, t);
      xv = ld2<V>(x, t);
      rv = ld2<V>(r, t);
    }
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    rv.x -= alpha * qv.x;
    rv.y -= alpha * qv.y;
    st2<V>(x, t, xv);
    st2<V>(r, t, rv);
    if (rf) {  // the V-cycle's FP32 input, written on the way
      rf[2 * t] = (float)rv.x;
      rf[2 * t + 1] = (float)rv.y;
    }
    acc[0] += wt.x * rv.x * rv.x;
    acc2 += wt.y * rv.y * rv.y;
  }
  if (t0 == 0 && (n & 1)) {
    x[n - 1] += alpha * p[n - 1];
    r[n - 1] -= alpha * q[n - 1];
    if (rf) rf[n - 1] = (float)r[n - 1];
    acc[0] += (double)w[n - 1] * r[n - 1] * r[n - 1];
  }
  acc[0] += acc2;
  block_partials<1>(acc, partials, pstride);
}

void launch_fcg_xr(const Ctx &c, int64_t n, const double *rz, const double *pq, const double *w,
                   const double *p, const double *q, double *x, double *r, double *out,
                   hipStream_t s, const float *w32, float *rf, const XDefer &xq) {
  const bool al = aligned16(p) && aligned16(q) && aligned16(x) && aligned16(r);
  const XDev f = xdev<double>(xq);
  unsigned g = red_grid(n);
  int ps = 8;
  if (xq.on) {
    if (!(w32 && al && ((uintptr_t)w32 & 7) == 0) || (n & 1))
      fail(SEM_EINVAL, "FCG update: a deferred gather-scatter step needs aligned vectors");
    // one sum, so its partials pack densely: up to 4 kRedBlocks blocks (at
    // 2^24 nodes, 16 waves per SIMD over the launch against 4 at kRedBlocks),
    // with p, w, x and r streamed non-temporally
    g = std::max(1u, std::min(nb(n / 2, 256), 4u * kRedBlocks));
    ps = 1;
    hipLaunchKernelGGL((k_fcg_xr<std::true_type, float, std::true_type, true>), dim3(g),
                       dim3(256), 0, s, n, rz, pq, w32, p, q, x, r, rf, c.partials, ps, f);
  } else if (w32 && al && ((uintptr_t)w32 & 7) == 0)
    hipLaunchKernelGGL((k_fcg_xr<std::true_type, float>), dim3(g), dim3(256), 0, s, n, rz, pq,
                       w32, p, q, x, r, rf, c.partials, ps, f);
  else if (al && aligned16(w))
    hipLaunchKernelGGL((k_fcg_xr<std::true_type, double>), dim3(g), dim3(256), 0, s, n, rz, pq, w,
                       p, q, x, r, rf, c.partials, ps, f);
  else
    hipLaunchKernelGGL((k_fcg_xr<std::false_type, double>), dim3(g), dim3(256), 0, s, n, rz, pq,
                       w, p, q, x, r, rf, c.partials, ps, f);
  SEM_LAUNCH("k_fcg_xr");
  launch_finish(1, g, c.partials, out, s, ps);
}

void launch_wdots(const Ctx &c, int64_t n, const double *w, int nd, const double *const *a,
                  const double *const *b, double *out, hipStream_t s, const float *w32) {
  Ptr4 pa{}, pb{};
  for (int j = 0; j < nd; ++j) {
    pa.p[j] = a[j];
    pb.p[j] = b[j];
  }
  unsigned g = red_grid(n);
  bool al = true;
  for (int j = 0; j < nd; ++j) al = al && aligned16(a[j]) && aligned16(b[j]);
  if (nd < 1 || nd > 4) fail(SEM_EINVAL, "wdots: at most 4 products");
#define WD(ND, V, WT, W) hipLaunchKernelGGL((k_wdots<ND, V, WT>), dim3(g), dim3(256), 0, s, n, W, pa, pb, c.partials)
#define WD_ALL(V, WT, W)                                                     \
  do {                                                                       \
    if (nd == 1) WD(1, V, WT, W);                                            \
    else if (nd == 2) WD(2, V, WT, W);                                       \
    else if (nd == 3) WD(3, V, WT, W);                                       \
    else WD(4, V, WT, W);                                                    \
  } while (0)
  if (w32 && al && ((uintptr_t)w32 & 7) == 0)
    WD_ALL(std::true_type, float, w32);
  else if (al && aligned16(w))
    WD_ALL(std::true_type, double, w);
  else
    WD_ALL(std::false_type, double, w);
#undef WD_ALL
#undef WD
  SEM_LAUNCH("k_wdots");
  launch_finish(nd, g, c.partials, out, s);
}

// (r, z_j)_w for FP32 z_j (j < ND): the preconditioned residual of the mixed
// path is the exact FP64 widening of the V-cycle's FP32 output, so it is read
// in FP32; the pairing of k_wdots, over up to 8 kRedBlocks / ND blocks whose
// partials pack densely (stride ND); r, w and z_old are streamed
// non-temporally (z is read again by the p update that follows)
template <int ND, typename WT>
__global__ __launch_bounds__(256) void k_wdots_rz(int64_t n, const WT *__restrict__ w,
                                                  const double *__restrict__ r,
                                                  const float *__restrict__ z0,
                                                  const float *__restrict__ z1, double *partials) {
  double acc[ND], acc2[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] = acc2[j] = 0.0;
  const int64_t n2 = n / 2;
  const int64_t t0 = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t t = t0; t < n2; t += (int64_t)gridDim.x * blockDim.x) {
    const double2 wt = ld2n<true>(w, t);
    const double2 x = ld2n<true>(r, t);
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      const double2 y = j == 0 ? ld2n<false>(z0, t) : ld2n<true>(z1, t);
      acc[j] += wt.x * x.x * y.x;
      acc2[j] += wt.y * x.y * y.y;
    }
  }
  if (t0 == 0 && (n & 1)) {
    const float *zs[2] = {z0, z1};
#pragma unroll
    for (int j = 0; j < ND; ++j) acc[j] += (double)w[n - 1] * r[n - 1] * (double)zs[j][n - 1];
  }
#pragma unroll
  for (int j = 0; j < ND; ++j) acc[j] += acc2[j];
  block_partials<ND>(acc, partials, ND);
}

void launch_wdots_rz(const Ctx &c, int64_t n, const double *w, const float *w32, const double *r,
                     const float *z0, const float *z1, double *out, hipStream_t s) {
  const int nd = z1 ? 2 : 1;
  const unsigned g = std::max(1u, std::min(nb(n / 2, 256), 8u * kRedBlocks / nd));
  if (!aligned16(r) || ((uintptr_t)z0 & 7) || (z1 && ((uintptr_t)z1 & 7)))
    fail(SEM_EINVAL, "wdots_rz: misaligned vectors");
  if (w32 && ((uintptr_t)w32 & 7) == 0) {
    if (nd == 1)
      hipLaunchKernelGGL((k_wdots_rz<1, float>), dim3(g), dim3(256), 0, s, n, w32, r, z0, z1,
                         c.partials);
    else
      hipLaunchKernelGGL((k_wdots_rz<2, float>), dim3(g), dim3(256), 0, s, n, w32, r, z0, z1,
                         c.partials);
  } else {
    if (!aligned16(w)) fail(SEM_EINVAL, "wdots_rz: misaligned weights");
    if (nd == 1)
      hipLaunchKernelGGL((k_wdots_rz<1, double>), dim3(g), dim3(256), 0, s, n, w, r, z0, z1,
                         c.partials);
    else
      hipLaunchKernelGGL((k_wdots_rz<2, double>), dim3(g), dim3(256), 0, s, n, w, r, z0, z1,
                         c.partials);
  }
  SEM_LAUNCH("k_wdots_rz");
  launch_finish(nd, g, c.partials, out, s, nd);
}

// p = z + beta p (FP64 p; z in FP32 on the mixed path), beta from the device
// scalars: (r, z) / rz_old, or ((r, z) - (r, z_old)) / rz_old when flexible
// (two nodes per thread: z non-temporal, its last read; p stays cached for
// the product A p that follows)
template <typename ZT>
__global__ void k_zp(int64_t n, const ZT *__restrict__ z, const double *__restrict__ rzn,
                     const double *__restrict__ rzo, int flexible, double *__restrict__ p) {
  const int64_t t = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  const double beta = (flexible ? rzn[0] - rzn[1] : rzn[0]) / rzo[0];
  const double a = 1.0;
  if (2 * t + 1 < n) {
    const double2 zv = ld2n<true>(z, t);
    double2 pv = reinterpret_cast<const double2 *>(p)[t];
    pv.x = a * zv.x + beta * pv.x;
    pv.y = a * zv.y + beta * pv.y;
    reinterpret_cast<double2 *>(p)[t] = pv;
  } else if (2 * t < n) {
    p[2 * t] = a * (double)z[2 * t] + beta * p[2 * t];
  }
}
template <typename ZT>
void launch_zp(int64_t n, const ZT *z, const double *rzn, const double *rzo, bool flexible,
               double *p, hipStream_t s) {
  if (!aligned16(p) || ((uintptr_t)z & (2 * sizeof(ZT) - 1)))
    fail(SEM_EINVAL, "p update: misaligned vectors");
  hipLaunchKernelGGL(k_zp<ZT>, dim3(nb((n + 1) / 2, 256)), dim3(256), 0, s, n, z, rzn, rzo,
                     flexible ? 1 : 0, p);
  SEM_LAUNCH("k_zp");
}
template void launch_zp<float>(int64_t, const float *, const double *, const double *, bool,
                               double *, hipStream_t);
template void launch_zp<double>(int64_t, const double *, const double *, const double *, bool,
                                double *, hipStream_t);

// block of inner products <V_j, x>_w for j < k (k <= 8 per pass)
template <int KB>
__global__ __launch_bounds__(256) void k_mdot(int64_t n, const double *__restrict__ w,
                                              const double *__restrict__ V, int64_t ld,
                                              const double *__restrict__ x, double *partials) {
  double acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double wx = w[t] * x[t];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] += wx * V[j * ld + t];
  }
  block_partials<KB>(acc, partials);
}

void launch_mdot(const Ctx &c, int64_t n, const double *w, int k, const double *V, int64_t ld,
                 const double *x, double *out, hipStream_t s) {
  unsigned g = red_grid(n);
  for (int j0 = 0; j0 < k; j0 += 8) {
    int kb = k - j0 < 8 ? k - j0 : 8;
    const double *Vj = V + j0 * ld;
    double *o = out + j0;
#define MD(KB) hipLaunchKernelGGL(k_mdot<KB>, dim3(g), dim3(256), 0, s, n, w, Vj, ld, x, c.partials)
    switch (kb) {
      case 1: MD(1); break;
      case 2: MD(2); break;
      case 3: MD(3); break;
      case 4: MD(4); break;
      case 5: MD(5); break;
      case 6: MD(6); break;
      case 7: MD(7); break;
      case 8: MD(8); break;
    }
#undef MD
    SEM_LAUNCH("k_mdot");
    launch_finish(kb, g, c.partials, o, s);
  }
}

__global__ void k_mupdate(int64_t n, int k, const double *__restrict__ V, int64_t ld,
                          const double *__restrict__ h, double *__restrict__ x, double sign) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc += h[j] * V[j * ld + t];
  x[t] += sign * acc;
}

void launch_mupdate(int64_t n, int k, const double *V, int64_t ld, const double *h, double *x,
                    double sign, hipStream_t s) {
  hipLaunchKernelGGL(k_mupdate, dim3(nb(n, 256)), dim3(256), 0, s, n, k, V, ld, h, x, sign);
  SEM_LAUNCH("k_mupdate");
}

// ---------------------------------------------------------------------------
// coarse-grid Jacobi-PCG with every scalar kept on the device; each kernel is
// a no-op once `done` is set, so a fixed number of iterations can be enqueued
// ahead of the convergence test.
__global__ __launch_bounds__(256) void k_cpcg_init(int64_t n, const double *__restrict__ w,
                                                   const double *__restrict__ dinv,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ z, double *__restrict__ p,
                                                   double *partials, unsigned *counter,
                                                   DevScalars *sc, double tol2, int maxit) {
  double acc[2] = {0.0, 0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double rv = b[t];
    double zv = dinv[t] * rv;
    x[t] = 0.0;
    r[t] = rv;
    z[t] = zv;
    p[t] = zv;
    acc[0] += w[t] * rv * zv;
    acc[1] += w[t] * rv * rv;
  }
  if (last_block_sum<2>(acc, partials, counter) && threadIdx.x == 0) {
    sc->rz = acc[0];
    sc->rr = acc[1];
    sc->rr0 = acc[1];
    sc->tol2 = tol2;
    sc->maxit = maxit;
    sc->beta = 0.0;
    sc->iters = 0;
    sc->done = (acc[1] == 0.0 || maxit <= 0) ? 1 : 0;
  }
}

__global__ void k_cpcg_p(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                         const DevScalars *sc) {
  if (sc->done) return;
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) p[t] = z[t] + sc->beta * p[t];
}

__global__ __launch_bounds__(256) void k_cpcg_pq(int64_t n, const double *__restrict__ w,
                                                 const double *__restrict__ p,
                                                 const double *__restrict__ q, double *partials,
                                                 unsigned *counter, DevScalars *sc) {
  if (sc->done) return;
  double acc[1] = {0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    acc[0] += w[t] * p[t] * q[t];
  if (last_block_sum<1>(acc, partials, counter) && threadIdx.x == 0) {
    sc->pq = acc[0];
    sc->alpha = acc[0] > 0.0 ? sc->rz / acc[0] : 0.0;
    if (!(acc[0] > 0.0)) sc->done = 1;  // exact breakdown: the iterate is exact
  }
}

__global__ __launch_bounds__(256) void k_cpcg_update(int64_t n, const double *__restrict__ w,
                                                     const double *__restrict__ dinv,
                                                     double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ z,
                                                     const double *__restrict__ p,
                                                     const double *__restrict__ q, double *partials,
                                                     unsigned *counter, DevScalars *sc) {
  if (sc->done) return;
  const double alpha = sc->alpha;
  double acc[2] = {0.0, 0.0};
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    x[t] += alpha * p[t];
    double rv = r[t] - alpha * q[t];
    double zv = dinv[t] * rv;
    r[t] = rv;
    z[t] = zv;
    acc[0] += w[t] * rv * zv;
    acc[1] += w[t] * rv * rv;
  }
  if (last_block_sum<2>(acc, partials, counter) && threadIdx.x == 0) {
    sc->beta = sc->rz != 0.0 ? acc[0] / sc->rz : 0.0;
    sc->rz = acc[0];
    if (!(acc[0] > 0.0)) sc->done = 1;
    sc->rr = acc[1];
    sc->iters += 1;
    bool conv = sc->tol2 > 0.0 && acc[1] <= sc->tol2 * sc->rr0;
    if (conv || sc->iters >= sc->maxit || !(acc[1] == acc[1])) sc->done = 1;
  }
}

void launch_cpcg_init(const Ctx &c, const Level &L, double tol2, int maxit, hipStream_t s) {
  hipLaunchKernelGGL(k_cpcg_init, dim3(red_grid(L.nloc)), dim3(256), 0, s, L.nloc, L.w64, L.dinv64,
                     L.d_b, c.cx, c.cr, c.cz, c.cp, c.partials, c.counter, c.dsc, tol2, maxit);
  SEM_LAUNCH("k_cpcg_init");
}

void launch_cpcg_iteration(const Ctx &c, const Level &L, bool first, hipStream_t s) {
  if (!first) {
    hipLaunchKernelGGL(k_cpcg_p, dim3(nb(L.nloc, 256)), dim3(256), 0, s, L.nloc, c.cz, c.cp, c.dsc);
    SEM_LAUNCH("k_cpcg_p");
  }
  launch_ax<double>(L, c.cp, c.cq, s);
  launch_gs<double>(L, c.cq, s);
  hipLaunchKernelGGL(k_cpcg_pq, dim3(red_grid(L.nloc)), dim3(256), 0, s, L.nloc, L.w64, c.cp, c.cq,
                     c.partials, c.counter, c.dsc);
  SEM_LAUNCH("k_cpcg_pq");
  hipLaunchKernelGGL(k_cpcg_update, dim3(red_grid(L.nloc)), dim3(256), 0, s, L.nloc, L.w64,
                     L.dinv64, c.cx, c.cr, c.cz, c.cp, c.cq, c.partials, c.counter, c.dsc);
  SEM_LAUNCH("k_cpcg_update");
}

}  // namespace sem
