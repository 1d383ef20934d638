// Local SE stiffness action v = A_L u by tensor-product sum factorisation
// (Sec. 2.1; about 7 E (p+1)^3 reads and 12 E (p+1)^4 operations, Sec. 1):
//
//   g = (D_r u, D_s u, D_t u)      three 1D contractions with Dhat
//   h = G g                         3x3 symmetric factors (6 per point)
//   v = D_r^T h_r + D_s^T h_s + D_t^T h_t
//
// Layout: u, v E-vectors [E][N][N][N] (i fastest); G [E][6][N^3], or for
// the FP32 smoother optionally G16 [E][3][N^3] FP16 pairs with a power-of-two
// scale per element (12 instead of 24 bytes per point).
// Mapping: one (i, j) column per thread with the t-line (k) in registers, so
// only the r and s contractions go through LDS; N^2 threads per element, EPB
// elements per workgroup.  Every G entry, u and v value is touched once per
// launch: loads of a k-plane by the N^2 lanes of an element are contiguous.
#include "sem_internal.h"

namespace sem {

template <int N>
struct AxShape {
  static constexpr int NN = N * N;
  static constexpr int N3 = N * NN;
  static constexpr int EPB = NN >= 256 ? 1 : 256 / NN;     // elements per workgroup
  static constexpr int BS = ((EPB * NN + 63) / 64) * 64;   // whole wavefronts
  static constexpr int RS = (N % 2 == 0) ? N + 1 : N;      // padded LDS row stride
  static constexpr int PS = N * RS;                        // LDS plane stride
};

// Several right sides (nv > 1): the nv workgroups of one element group run on
// one XCD back to back, so the group's G comes from HBM once and from L2 for
// the other right sides.
__device__ inline unsigned rhs_block(int nv, int &vec) {
  if (nv == 1) {
    vec = 0;
    return blockIdx.x;
  }
  return split_rhs(xcd_block(), nv, vec);
}

// FP16 geometric factors (FP32 smoother, geom_prec = SEM_F16): pairs
// G16[e][c][point] = (G_2c, G_2c+1) scaled by 2^s per element; the element's
// result is multiplied by gsc[e] = 2^-s, which commutes with FP32 rounding.
__device__ __forceinline__ float half_lo(uint32_t w) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}
__device__ __forceinline__ float half_hi(uint32_t w) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// GH: the factors come from G16 / gsc instead of G (FP32 only)
template <int N, typename T, bool GH>
__global__ __launch_bounds__(AxShape<N>::BS) void k_ax(int64_t E, const T *__restrict__ u,
                                                       const T *__restrict__ G,
                                                       const T *__restrict__ Dg,
                                                       T *__restrict__ v, int nv,
                                                       const uint32_t *__restrict__ G16,
                                                       const float *__restrict__ gsc) {
  using S = AxShape<N>;
  constexpr int NN = S::NN, N3 = S::N3, EPB = S::EPB, RS = S::RS, PS = S::PS;
  __shared__ T sD[NN];
  __shared__ T s_a[EPB][N * PS];
  __shared__ T s_b[EPB][N * PS];

  const int tid = threadIdx.x;
  const int le = tid / NN;
  const int ij = tid - le * NN;
  const int i = ij % N, j = ij / N;
  int vec;
  const int64_t e = (int64_t)rhs_block(nv, vec) * EPB + le;
  u += (int64_t)vec * E * N3;
  v += (int64_t)vec * E * N3;
  const bool active = le < EPB && e < E;

  for (int t = tid; t < NN; t += S::BS) sD[t] = Dg[t];

  // phase 1: the element's u into registers (t-lines) and LDS (planes)
  T uk[N];
  if (active) {
    const T *ue = u + e * N3 + ij;
#pragma unroll
    for (int k = 0; k < N; ++k) uk[k] = ue[k * NN];
#pragma unroll
    for (int k = 0; k < N; ++k) s_a[le][k * PS + j * RS + i] = uk[k];
  }
  __syncthreads();

  // phase 2: r and s derivatives from LDS
  T Di[N], Dj[N], ur[N], us[N];
  if (active) {
#pragma unroll
    for (int l = 0; l < N; ++l) {
      Di[l] = sD[i * N + l];
      Dj[l] = sD[j * N + l];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      T a = 0, b = 0;
#pragma unroll
      for (int l = 0; l < N; ++l) {
        a += Di[l] * s_a[le][k * PS + j * RS + l];
        b += Dj[l] * s_a[le][k * PS + l * RS + i];
      }
      ur[k] = a;
      us[k] = b;
    }
  }
  __syncthreads();

  // phase 3: t derivative in registers, h = G g; h_r, h_s to LDS, h_t stays
  T wt[N];
  if (active) {
    const T *Ge = GH ? nullptr : G + e * 6 * N3 + ij;
    const uint32_t *He = GH ? G16 + e * 3 * N3 + ij : nullptr;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      T ut = 0;
#pragma unroll
      for (int l = 0; l < N; ++l) ut += sD[k * N + l] * uk[l];
      T g0, g1, g2, g3, g4, g5;
      if constexpr (GH) {
        const uint32_t h01 = He[0 * N3 + k * NN], h23 = He[1 * N3 + k * NN];
        const uint32_t h45 = He[2 * N3 + k * NN];
        g0 = half_lo(h01); g1 = half_hi(h01);
        g2 = half_lo(h23); g3 = half_hi(h23);
        g4 = half_lo(h45); g5 = half_hi(h45);
      } else {
        g0 = Ge[0 * N3 + k * NN]; g1 = Ge[1 * N3 + k * NN]; g2 = Ge[2 * N3 + k * NN];
        g3 = Ge[3 * N3 + k * NN]; g4 = Ge[4 * N3 + k * NN]; g5 = Ge[5 * N3 + k * NN];
      }
      s_a[le][k * PS + j * RS + i] = g0 * ur[k] + g1 * us[k] + g2 * ut;
      s_b[le][k * PS + j * RS + i] = g1 * ur[k] + g3 * us[k] + g4 * ut;
      wt[k] = g2 * ur[k] + g4 * us[k] + g5 * ut;
    }
  }
  __syncthreads();
  if (!active) return;

  // phase 4: v = D_r^T h_r + D_s^T h_s + D_t^T h_t
#pragma unroll
  for (int l = 0; l < N; ++l) {
    Di[l] = sD[l * N + i];
    Dj[l] = sD[l * N + j];
  }
  T *ve = v + e * N3 + ij;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T acc = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      acc += Di[l] * s_a[le][k * PS + j * RS + l];
      acc += Dj[l] * s_b[le][k * PS + l * RS + i];
      acc += sD[l * N + k] * wt[l];
    }
    if constexpr (GH) acc *= gsc[e];
    ve[k * NN] = acc;
  }
}

// p = 7 (N = 8): one element per wavefront, lane (i, j) of the 8x8 slab.  The
// element is swept plane by plane; each k-plane of u, h_r and h_s lives in LDS
// only while it is used, and the transposed r/s contractions of plane k run as
// soon as that plane's h is known, so the only whole-element state is the
// t-line of u and of the output (registers).  Plane exchanges are within one
// wavefront: LDS operations of a wavefront complete in issue order, and the
// wave barriers keep the compiler from moving LDS accesses across phases.
// streaming loads/stores: NT = true marks them non-temporal (no reuse)
template <bool NT, typename T>
__device__ __forceinline__ T ld(const T *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st(T *p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// XF: the four elements of a workgroup are consecutive along x (nex a multiple
// of 4), and the copies on their three shared x-faces are summed here, in LDS,
// before the store (the first pass of the direction-by-direction gather-scatter
// for those faces; the faces between workgroups and the Dirichlet x-faces are
// left to the gather-scatter).  Each pair is summed as (p-face + 0-face), the
// order the gather-scatter uses.
//
// dotp (may be null; one right side): element e's share of u^T A_L u, the sum
// of u times its unassembled product over the element's points, goes to
// dotp[e].  For u consistent and zero on Dirichlet nodes the element shares add
// up to (u, Au) over the unique free nodes, the product the gather-scatter
// completes (the copies of a node sum to its assembled row).
//
// GH (FP32 only): the factors come as FP16 pairs from G16, and the element's
// result is multiplied by gsc[e] before the x-face sums and the store.

template <typename T, bool NT, bool XF, bool GH = false>
__device__ __forceinline__ void ax8_body(int64_t E, const T *__restrict__ u,
                                         const T *__restrict__ G, const T *__restrict__ Dg,
                                         T *__restrict__ v, int nv, T *sD, T (*sU)[72],
                                         T (*sR)[72], T (*sS)[72], double *dotp = nullptr,
                                         const uint32_t *__restrict__ G16 = nullptr,
                                         const float *__restrict__ gsc = nullptr) {
  constexpr int N = 8, NN = 64, N3 = 512, RS = 9;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 7, j = lane >> 3;
  if (threadIdx.x < NN) sD[threadIdx.x] = Dg[threadIdx.x];
  __syncthreads();
  int vec;
  const int64_t e = (int64_t)rhs_block(nv, vec) * 4 + w;
  if (e >= E) return;
  u += (int64_t)vec * E * N3;
  v += (int64_t)vec * E * N3;

  T Di[N], Dj[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    Di[l] = sD[i * N + l];
    Dj[l] = sD[j * N + l];
  }
  const T *ue = u + e * N3 + lane;
  const T *Ge = GH ? nullptr : G + e * 6 * N3 + lane;
  const uint32_t *He = GH ? G16 + e * 3 * N3 + lane : nullptr;
  T uk[N], acc[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    uk[k] = ld<NT>(ue + k * NN);
    acc[k] = T(0);
  }
  T *su = sU[w], *sr = sR[w], *ss = sS[w];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T g0, g1, g2, g3, g4, g5;
    if constexpr (GH) {
      const uint32_t h01 = ld<NT>(He + 0 * N3 + k * NN), h23 = ld<NT>(He + 1 * N3 + k * NN);
      const uint32_t h45 = ld<NT>(He + 2 * N3 + k * NN);
      g0 = half_lo(h01); g1 = half_hi(h01);
      g2 = half_lo(h23); g3 = half_hi(h23);
      g4 = half_lo(h45); g5 = half_hi(h45);
    } else {
      g0 = ld<NT>(Ge + 0 * N3 + k * NN); g1 = ld<NT>(Ge + 1 * N3 + k * NN);
      g2 = ld<NT>(Ge + 2 * N3 + k * NN); g3 = ld<NT>(Ge + 3 * N3 + k * NN);
      g4 = ld<NT>(Ge + 4 * N3 + k * NN); g5 = ld<NT>(Ge + 5 * N3 + k * NN);
    }
    su[j * RS + i] = uk[k];
    __builtin_amdgcn_wave_barrier();
    T ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      ur += Di[l] * su[j * RS + l];
      us += Dj[l] * su[l * RS + i];
      ut += Dg[k * N + l] * uk[l];
    }
    const T hr = g0 * ur + g1 * us + g2 * ut;
    const T hs = g1 * ur + g3 * us + g4 * ut;
    const T ht = g2 * ur + g4 * us + g5 * ut;
    __builtin_amdgcn_wave_barrier();
    sr[j * RS + i] = hr;
    ss[j * RS + i] = hs;
    __builtin_amdgcn_wave_barrier();
    T a = 0;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      a += sD[l * N + i] * sr[j * RS + l];
      a += sD[l * N + j] * ss[l * RS + i];
      acc[l] += Dg[k * N + l] * ht;  // D_t^T: v[l] += D[k][l] h_t[k]
    }
    acc[k] += a;
    __builtin_amdgcn_wave_barrier();
  }
  if constexpr (GH) {
    const float sc = gsc[e];
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k] *= sc;
  }
  if (dotp) {  // fixed order: the lane's k-line, then a butterfly over the wave
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) d += (double)uk[k] * (double)acc[k];
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) d += __shfl_xor(d, sh, 64);
    if (lane == 0) dotp[e] = d;
  }
  if constexpr (XF) {  // every wave of the block is live (E is a multiple of 4)
    if (i == 0) {
#pragma unroll
      for (int k = 0; k < N; ++k) sr[k * N + j] = acc[k];
    }
    if (i == N - 1) {
#pragma unroll
      for (int k = 0; k < N; ++k) ss[k * N + j] = acc[k];
    }
    __syncthreads();
    if (i == N - 1 && w < 3) {
#pragma unroll
      for (int k = 0; k < N; ++k) acc[k] = sS[w][k * N + j] + sR[w + 1][k * N + j];
    }
    if (i == 0 && w > 0) {
#pragma unroll
      for (int k = 0; k < N; ++k) acc[k] = sS[w - 1][k * N + j] + sR[w][k * N + j];
    }
  }
  T *ve = v + e * N3 + lane;
#pragma unroll
  for (int k = 0; k < N; ++k) st<NT>(ve + k * NN, acc[k]);
}

// register budgets: FP64 at 4 waves/SIMD, FP32 at 6
template <bool NT, bool XF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_ax8_f64(
    int64_t E, const double *__restrict__ u, const double *__restrict__ G,
    const double *__restrict__ Dg, double *__restrict__ v, int nv, double *dotp) {
  __shared__ double sD[64], sU[4][72], sR[4][72], sS[4][72];
  ax8_body<double, NT, XF>(E, u, G, Dg, v, nv, sD, sU, sR, sS, dotp);
}
template <bool NT, bool XF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_ax8_f32(
    int64_t E, const float *__restrict__ u, const float *__restrict__ G,
    const float *__restrict__ Dg, float *__restrict__ v, int nv) {
  __shared__ float sD[64], sU[4][72], sR[4][72], sS[4][72];
  ax8_body<float, NT, XF>(E, u, G, Dg, v, nv, sD, sU, sR, sS);
}

template <bool NT, bool XF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_ax8_f32h(
    int64_t E, const float *__restrict__ u, const uint32_t *__restrict__ G16,
    const float *__restrict__ gsc, const float *__restrict__ Dg, float *__restrict__ v, int nv) {
  __shared__ float sD[64], sU[4][72], sR[4][72], sS[4][72];
  ax8_body<float, NT, XF, true>(E, u, nullptr, Dg, v, nv, sD, sU, sR, sS, nullptr, G16, gsc);
}

template <typename T, bool XF>
static void ax8_launch(const Level &L, const T *u, T *v, const T *G, const T *D, int nv,
                       hipStream_t s, double *dotp) {
  // several right sides share G through L2: plain loads (non-temporal ones would bypass it)
  const dim3 grid((unsigned)((L.E + 3) / 4 * nv));
  const bool nt = L.ax_variant == 2 && nv == 1;
  if constexpr (sizeof(T) == 8) {
    if (nt)
      hipLaunchKernelGGL((k_ax8_f64<true, XF>), grid, dim3(256), 0, s, L.E, u, G, D, v, nv, dotp);
    else
      hipLaunchKernelGGL((k_ax8_f64<false, XF>), grid, dim3(256), 0, s, L.E, u, G, D, v, nv,
                         dotp);
  } else if (L.G16) {  // FP16 factors
    if (nt)
      hipLaunchKernelGGL((k_ax8_f32h<true, XF>), grid, dim3(256), 0, s, L.E, u, L.G16, L.gscale,
                         D, v, nv);
    else
      hipLaunchKernelGGL((k_ax8_f32h<false, XF>), grid, dim3(256), 0, s, L.E, u, L.G16, L.gscale,
                         D, v, nv);
  } else {
    if (nt)
      hipLaunchKernelGGL((k_ax8_f32<true, XF>), grid, dim3(256), 0, s, L.E, u, G, D, v, nv);
    else
      hipLaunchKernelGGL((k_ax8_f32<false, XF>), grid, dim3(256), 0, s, L.E, u, G, D, v, nv);
  }
  SEM_LAUNCH("k_ax8");
}

template <typename T, int N>
static void ax_n(const Level &L, const T *u, T *v, const T *G, const T *D, int nv, bool xf,
                 hipStream_t s, double *dotp) {
  if constexpr (N == 8) {
    if (L.ax_variant >= 1) {
      if (xf)
        ax8_launch<T, true>(L, u, v, G, D, nv, s, dotp);
      else
        ax8_launch<T, false>(L, u, v, G, D, nv, s, dotp);
      return;
    }
  }
  if (xf) fail(SEM_EINVAL, "x-face summation in Ax needs the p = 7 one-wave kernel");
  using S = AxShape<N>;
  unsigned grid = (unsigned)((L.E + S::EPB - 1) / S::EPB * nv);
  if constexpr (sizeof(T) == 4) {
    if (L.G16) {  // FP16 factors
      hipLaunchKernelGGL((k_ax<N, float, true>), dim3(grid), dim3(S::BS), 0, s, L.E, u, G, D, v,
                         nv, (const uint32_t *)L.G16, (const float *)L.gscale);
      SEM_LAUNCH("k_ax");
      return;
    }
  }
  hipLaunchKernelGGL((k_ax<N, T, false>), dim3(grid), dim3(S::BS), 0, s, L.E, u, G, D, v, nv,
                     (const uint32_t *)nullptr, (const float *)nullptr);
  SEM_LAUNCH("k_ax");
}

bool ax_sums_x_faces(const Level &L) {
  return L.gs_struct && L.xfuse && L.N == 8 && L.ax_variant >= 1 && L.nex % 4 == 0;
}

bool ax_forms_dot(const Level &L, int nv) { return L.N == 8 && L.ax_variant >= 1 && nv == 1; }

template <typename T>
void launch_ax(const Level &L, const T *u, T *v, hipStream_t s, int nv, bool xf, double *dotp) {
  if (nv < 1) fail(SEM_EINVAL, "Ax: no right side");
  if (xf && !ax_sums_x_faces(L)) fail(SEM_EINVAL, "Ax: x-face summation not available here");
  if (dotp && (sizeof(T) != 8 || !ax_forms_dot(L, nv)))
    fail(SEM_EINVAL, "Ax: the element shares of (u, Au) need the FP64 p = 7 one-wave kernel");
  const T *G;
  const T *D;
  if constexpr (sizeof(T) == 8) {
    G = (const T *)L.G64;
    D = (const T *)L.D64;
  } else {
    G = (const T *)L.G32;
    D = (const T *)L.D32;
  }
  if (!G || !D) fail(SEM_EINVAL, "geometric factors of this precision were not built");
  switch (L.N) {
    case 2: ax_n<T, 2>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 3: ax_n<T, 3>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 4: ax_n<T, 4>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 5: ax_n<T, 5>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 6: ax_n<T, 6>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 7: ax_n<T, 7>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 8: ax_n<T, 8>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 9: ax_n<T, 9>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 10: ax_n<T, 10>(L, u, v, G, D, nv, xf, s, dotp); break;
    case 11: ax_n<T, 11>(L, u, v, G, D, nv, xf, s, dotp); break;
    default: fail(SEM_EUNSUPPORTED, "Ax: unsupported degree");
  }
}
template void launch_ax<double>(const Level &, const double *, double *, hipStream_t, int, bool,
                                double *);
template void launch_ax<float>(const Level &, const float *, float *, hipStream_t, int, bool,
                               double *);

// diag(A^e) per point: only q' on the r-, s- or t-line through q contribute, and
// the cross terms only at q' = q.
__global__ void k_diag(int64_t E, int N, const double *__restrict__ G, const double *__restrict__ D,
                       double *__restrict__ d) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int N3 = N * N * N;
  if (t >= E * N3) return;
  int64_t e = t / N3;
  int q = (int)(t - e * N3);
  int i = q % N, j = (q / N) % N, k = q / (N * N);
  const double *Ge = G + e * 6 * N3;
  double acc = 0;
  for (int l = 0; l < N; ++l) {
    double a = D[l * N + i], b = D[l * N + j], c = D[l * N + k];
    acc += a * a * Ge[0 * N3 + (k * N + j) * N + l];
    acc += b * b * Ge[3 * N3 + (k * N + l) * N + i];
    acc += c * c * Ge[5 * N3 + (l * N + j) * N + i];
  }
  double di = D[i * N + i], dj = D[j * N + j], dk = D[k * N + k];
  acc += 2 * di * dj * Ge[1 * N3 + q] + 2 * di * dk * Ge[2 * N3 + q] + 2 * dj * dk * Ge[4 * N3 + q];
  d[t] = acc;
}

void launch_diag(const Level &L, double *d, hipStream_t s) {
  hipLaunchKernelGGL(k_diag, dim3((unsigned)((L.nloc + 255) / 256)), dim3(256), 0, s, L.E, L.N,
                     L.G64, L.D64, d);
  SEM_LAUNCH("k_diag");
}

}  // namespace sem
