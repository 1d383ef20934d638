// p-multigrid transfers (Sec. 2.2.2, Algorithm 1, "coarsen" and "prolongate").
//
// P interpolates the coarse cardinal basis to the fine GLL nodes element by
// element, P = J (x) J (x) J with J[i][j] = h^c_j(xi^f_i); a continuous coarse
// field stays continuous, so the fine E-vector comes out consistent.
// P^T (on global vectors) = assemble_c o (J^T (x) J^T (x) J^T) o (1/mult_f):
// the consistent fine residual is split among its copies, contracted, then
// summed over shared coarse nodes (QQ^T) and masked by the caller.
#include "sem_internal.h"

namespace sem {

constexpr int kTN = 11;  // largest N handled (p <= 10)

// NF, NC > 0: sizes fixed at compile time (the loops unroll, 256 threads);
// 0: taken from the arguments
template <typename T, int NF = 0, int NC = 0>
__global__ __launch_bounds__(256) void k_prolong(int Nf_, int Nc_, const T *__restrict__ J,
                                                 const T *__restrict__ xc, T *__restrict__ xf) {
  __shared__ T sJ[kTN * kTN];
  __shared__ T a[kTN * kTN * kTN];
  __shared__ T b[kTN * kTN * kTN];
  const int Nf = NF ? NF : Nf_, Nc = NC ? NC : Nc_;
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x, bs = NF ? 256 : (int)blockDim.x;
  const int Nc3 = Nc * Nc * Nc, Nf3 = Nf * Nf * Nf;
  xc += blockIdx.y * (int64_t)gridDim.x * Nc3;  // right side blockIdx.y
  xf += blockIdx.y * (int64_t)gridDim.x * Nf3;
  // two neighbouring fine points per thread when the element has 512: their
  // old values are requested first (streamed, no reuse) and arrive while the
  // contractions run
  constexpr bool two = NF > 0 && NF * NF * NF == 2 * 256;
  using T2 = T __attribute__((ext_vector_type(2)));
  T2 *dst = nullptr;
  T2 old{};
  if constexpr (two) {
    dst = reinterpret_cast<T2 *>(xf + e * Nf3 + 2 * tid);
    old = __builtin_nontemporal_load(dst);
  }
  for (int t = tid; t < Nf * Nc; t += bs) sJ[t] = J[t];
  for (int t = tid; t < Nc3; t += bs) a[t] = xc[e * Nc3 + t];
  __syncthreads();
  // b[c][bb][i] = sum_a J[i][a] x[c][bb][a]
  for (int t = tid; t < Nc * Nc * Nf; t += bs) {
    int i = t % Nf, cb = t / Nf;
    T s = 0;
#pragma unroll
    for (int q = 0; q < Nc; ++q) s += sJ[i * Nc + q] * a[cb * Nc + q];
    b[t] = s;
  }
  __syncthreads();
  // a[c][j][i] = sum_bb J[j][bb] b[c][bb][i]
  for (int t = tid; t < Nc * Nf * Nf; t += bs) {
    int i = t % Nf, j = (t / Nf) % Nf, c = t / (Nf * Nf);
    T s = 0;
#pragma unroll
    for (int q = 0; q < Nc; ++q) s += sJ[j * Nc + q] * b[(c * Nc + q) * Nf + i];
    a[t] = s;
  }
  __syncthreads();
  // xf[k][j][i] += sum_c J[k][c] a[c][j][i]
  if constexpr (two) {
    // the thread's two points share k (NF^2 is even), one 2-wide store
    const int t = 2 * tid, ji = t % (NF * NF), k = t / (NF * NF);
    T s0 = 0, s1 = 0;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      s0 += sJ[k * NC + q] * a[q * NF * NF + ji];
      s1 += sJ[k * NC + q] * a[q * NF * NF + ji + 1];
    }
    old[0] += s0;
    old[1] += s1;
    __builtin_nontemporal_store(old, dst);
  } else {
    for (int t = tid; t < Nf3; t += bs) {
      int ji = t % (Nf * Nf), k = t / (Nf * Nf);
      T s = 0;
#pragma unroll
      for (int q = 0; q < Nc; ++q) s += sJ[k * Nc + q] * a[q * Nf * Nf + ji];
      xf[e * Nf3 + t] += s;
    }
  }
}

template <typename T, int NF = 0, int NC = 0>
__global__ __launch_bounds__(256) void k_restrict(int Nf_, int Nc_, const T *__restrict__ J,
                                                  const T *__restrict__ w, const T *__restrict__ rf,
                                                  const T *__restrict__ bf, T *__restrict__ rc) {
  __shared__ T sJ[kTN * kTN];
  __shared__ T a[kTN * kTN * kTN];
  __shared__ T b[kTN * kTN * kTN];
  const int Nf = NF ? NF : Nf_, Nc = NC ? NC : Nc_;
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x, bs = NF ? 256 : (int)blockDim.x;
  const int Nc3 = Nc * Nc * Nc, Nf3 = Nf * Nf * Nf;
  rf += blockIdx.y * (int64_t)gridDim.x * Nf3;  // right side blockIdx.y
  rc += blockIdx.y * (int64_t)gridDim.x * Nc3;
  for (int t = tid; t < Nf * Nc; t += bs) sJ[t] = J[t];
  if (bf) bf += blockIdx.y * (int64_t)gridDim.x * Nf3;
  if constexpr (NF > 0 && NF * NF * NF == 2 * 256) {
    // two neighbouring points per thread, 2-wide loads
    using T2 = T __attribute__((ext_vector_type(2)));
    const int64_t o = e * Nf3 + 2 * tid;
    const T2 wv = *reinterpret_cast<const T2 *>(w + o);
    const T2 rv = *reinterpret_cast<const T2 *>(rf + o);
    const T2 res = bf ? *reinterpret_cast<const T2 *>(bf + o) - rv : rv;  // b - A x on the way in
    a[2 * tid] = wv[0] * res[0];
    a[2 * tid + 1] = wv[1] * res[1];
  } else if (bf) {  // residual b - A x formed on the way in
    for (int t = tid; t < Nf3; t += bs) a[t] = w[e * Nf3 + t] * (bf[e * Nf3 + t] - rf[e * Nf3 + t]);
  } else {
    for (int t = tid; t < Nf3; t += bs) a[t] = w[e * Nf3 + t] * rf[e * Nf3 + t];
  }
  __syncthreads();
  // b[k][j][aa] = sum_i J[i][aa] r[k][j][i]
  for (int t = tid; t < Nf * Nf * Nc; t += bs) {
    int aa = t % Nc, kj = t / Nc;
    T s = 0;
#pragma unroll
    for (int q = 0; q < Nf; ++q) s += sJ[q * Nc + aa] * a[kj * Nf + q];
    b[t] = s;
  }
  __syncthreads();
  // a[k][bb][aa] = sum_j J[j][bb] b[k][j][aa]
  for (int t = tid; t < Nf * Nc * Nc; t += bs) {
    int aa = t % Nc, bb = (t / Nc) % Nc, k = t / (Nc * Nc);
    T s = 0;
#pragma unroll
    for (int q = 0; q < Nf; ++q) s += sJ[q * Nc + bb] * b[(k * Nf + q) * Nc + aa];
    a[t] = s;
  }
  __syncthreads();
  // rc[c][bb][aa] = sum_k J[k][c] a[k][bb][aa]
  for (int t = tid; t < Nc3; t += bs) {
    int ba = t % (Nc * Nc), c = t / (Nc * Nc);
    T s = 0;
#pragma unroll
    for (int q = 0; q < Nf; ++q) s += sJ[q * Nc + c] * a[q * Nc * Nc + ba];
    rc[e * Nc3 + t] = s;
  }
}

// Small elements (NF^3 <= 64, e.g. p = 3 -> 1): one element per wavefront,
// four per workgroup, the same contractions and summation order as above;
// E is passed for the right-side stride (gridDim.x counts workgroups).
template <typename T, int NF, int NC>
__global__ __launch_bounds__(256) void k_prolong_w(int64_t E, const T *__restrict__ J,
                                                   const T *__restrict__ xc, T *__restrict__ xf) {
  static_assert(NF * NF * NF <= 64, "one element per wavefront");
  constexpr int Nc3 = NC * NC * NC, Nf3 = NF * NF * NF;
  __shared__ T sJ[NF * NC];
  __shared__ T a[4][64];
  __shared__ T b[4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + w;
  const bool act = e < E;
  xc += blockIdx.y * E * Nc3;  // right side blockIdx.y
  xf += blockIdx.y * E * Nf3;
  if (threadIdx.x < NF * NC) sJ[threadIdx.x] = J[threadIdx.x];
  if (act && l < Nc3) a[w][l] = xc[e * Nc3 + l];
  __syncthreads();
  if (l < NC * NC * NF) {  // b[c][bb][i] = sum_a J[i][a] x[c][bb][a]
    const int i = l % NF, cb = l / NF;
    T s = 0;
#pragma unroll
    for (int q = 0; q < NC; ++q) s += sJ[i * NC + q] * a[w][cb * NC + q];
    b[w][l] = s;
  }
  __syncthreads();
  if (l < NC * NF * NF) {  // a[c][j][i] = sum_bb J[j][bb] b[c][bb][i]
    const int i = l % NF, j = (l / NF) % NF, c = l / (NF * NF);
    T s = 0;
#pragma unroll
    for (int q = 0; q < NC; ++q) s += sJ[j * NC + q] * b[w][(c * NC + q) * NF + i];
    a[w][l] = s;
  }
  __syncthreads();
  if (act && l < Nf3) {  // xf[k][j][i] += sum_c J[k][c] a[c][j][i]
    const int ji = l % (NF * NF), k = l / (NF * NF);
    T s = 0;
#pragma unroll
    for (int q = 0; q < NC; ++q) s += sJ[k * NC + q] * a[w][q * NF * NF + ji];
    xf[e * Nf3 + l] += s;
  }
}

template <typename T, int NF, int NC>
__global__ __launch_bounds__(256) void k_restrict_w(int64_t E, const T *__restrict__ J,
                                                    const T *__restrict__ wt,
                                                    const T *__restrict__ rf,
                                                    const T *__restrict__ bf, T *__restrict__ rc) {
  static_assert(NF * NF * NF <= 64, "one element per wavefront");
  constexpr int Nc3 = NC * NC * NC, Nf3 = NF * NF * NF;
  __shared__ T sJ[NF * NC];
  __shared__ T a[4][64];
  __shared__ T b[4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 4 + w;
  const bool act = e < E;
  rf += blockIdx.y * E * Nf3;  // right side blockIdx.y
  rc += blockIdx.y * E * Nc3;
  if (bf) bf += blockIdx.y * E * Nf3;
  if (threadIdx.x < NF * NC) sJ[threadIdx.x] = J[threadIdx.x];
  if (act && l < Nf3) {
    const int64_t o = e * Nf3 + l;
    a[w][l] = bf ? wt[o] * (bf[o] - rf[o]) : wt[o] * rf[o];  // b - A x on the way in
  }
  __syncthreads();
  if (l < NF * NF * NC) {  // b[k][j][aa] = sum_i J[i][aa] r[k][j][i]
    const int aa = l % NC, kj = l / NC;
    T s = 0;
#pragma unroll
    for (int q = 0; q < NF; ++q) s += sJ[q * NC + aa] * a[w][kj * NF + q];
    b[w][l] = s;
  }
  __syncthreads();
  if (l < NF * NC * NC) {  // a[k][bb][aa] = sum_j J[j][bb] b[k][j][aa]
    const int aa = l % NC, bb = (l / NC) % NC, k = l / (NC * NC);
    T s = 0;
#pragma unroll
    for (int q = 0; q < NF; ++q) s += sJ[q * NC + bb] * b[w][(k * NF + q) * NC + aa];
    a[w][l] = s;
  }
  __syncthreads();
  if (act && l < Nc3) {  // rc[c][bb][aa] = sum_k J[k][c] a[k][bb][aa]
    const int ba = l % (NC * NC), c = l / (NC * NC);
    T s = 0;
#pragma unroll
    for (int q = 0; q < NF; ++q) s += sJ[q * NC + c] * a[w][q * NC * NC + ba];
    rc[e * Nc3 + l] = s;
  }
}

static int transfer_threads(int Nf) {
  int n = Nf * Nf * Nf;
  int t = ((n + 63) / 64) * 64;
  return t > 256 ? 256 : t;
}

// compile-time sizes for the pairs of the usual schedules (fine N >= 6, so
// 256 threads), the generic kernel otherwise
#define SEM_TRANSFER_PAIRS(X) X(8, 4) X(6, 4) X(10, 6) X(10, 8) X(8, 6)

template <typename T>
void launch_prolong(const Level &F, const Level &C, const T *xc, T *xf, hipStream_t s, int nv) {
  const T *J = sizeof(T) == 8 ? (const T *)F.J64 : (const T *)F.J32;
  const dim3 grid((unsigned)F.E, (unsigned)nv);
#define SEM_PROLONG_CASE(NF, NC)                                                             \
  if (F.N == NF && C.N == NC) {                                                              \
    hipLaunchKernelGGL((k_prolong<T, NF, NC>), grid, dim3(256), 0, s, F.N, C.N, J, xc, xf); \
    SEM_LAUNCH("k_prolong");                                                                 \
    return;                                                                                  \
  }
  SEM_TRANSFER_PAIRS(SEM_PROLONG_CASE)
#undef SEM_PROLONG_CASE
  if (F.N == 4 && C.N == 2) {
    const dim3 gw((unsigned)((F.E + 3) / 4), (unsigned)nv);
    hipLaunchKernelGGL((k_prolong_w<T, 4, 2>), gw, dim3(256), 0, s, F.E, J, xc, xf);
    SEM_LAUNCH("k_prolong");
    return;
  }
  hipLaunchKernelGGL(k_prolong<T>, grid, dim3(transfer_threads(F.N)), 0, s, F.N, C.N, J, xc, xf);
  SEM_LAUNCH("k_prolong");
}

template <typename T>
void launch_restrict(const Level &F, const Level &C, const T *rf, T *rc, hipStream_t s, int nv,
                     const T *bf) {
  const T *J = sizeof(T) == 8 ? (const T *)F.J64 : (const T *)F.J32;
  const T *w = sizeof(T) == 8 ? (const T *)F.w64 : (const T *)F.w32;
  const dim3 grid((unsigned)F.E, (unsigned)nv);
#define SEM_RESTRICT_CASE(NF, NC)                                                          \
  if (F.N == NF && C.N == NC) {                                                            \
    hipLaunchKernelGGL((k_restrict<T, NF, NC>), grid, dim3(256), 0, s, F.N, C.N, J, w, rf, \
                       bf, rc);                                                            \
    SEM_LAUNCH("k_restrict");                                                              \
    return;                                                                                \
  }
  SEM_TRANSFER_PAIRS(SEM_RESTRICT_CASE)
#undef SEM_RESTRICT_CASE
  if (F.N == 4 && C.N == 2) {
    const dim3 gw((unsigned)((F.E + 3) / 4), (unsigned)nv);
    hipLaunchKernelGGL((k_restrict_w<T, 4, 2>), gw, dim3(256), 0, s, F.E, J, w, rf, bf, rc);
    SEM_LAUNCH("k_restrict");
    return;
  }
  hipLaunchKernelGGL(k_restrict<T>, grid, dim3(transfer_threads(F.N)), 0, s, F.N, C.N, J, w, rf,
                     bf, rc);
  SEM_LAUNCH("k_restrict");
}
#undef SEM_TRANSFER_PAIRS

template void launch_prolong<double>(const Level &, const Level &, const double *, double *,
                                     hipStream_t, int);
template void launch_prolong<float>(const Level &, const Level &, const float *, float *,
                                    hipStream_t, int);
template void launch_restrict<double>(const Level &, const Level &, const double *, double *,
                                      hipStream_t, int, const double *);
template void launch_restrict<float>(const Level &, const Level &, const float *, float *,
                                     hipStream_t, int, const float *);

}  // namespace sem
