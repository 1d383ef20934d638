// Overlapping Schwarz smoother with fast-diagonalisation local solves
// (Sec. 2.2.2, eqs. 4-9).
//
// Setup, per element, level and direction: the element is approximated by a
// box whose length along r is the mean of its four r-edges; the 1D stiffness
// (2/L) Dhat^T W Dhat and mass (L/2) W are assembled over the element and its
// two neighbours and restricted to the extended grid (left neighbour's node
// p-1, own nodes 0..p, right neighbour's node 1), so pbar = p+3.  Nodes with no
// neighbour (domain boundary), and the element's own boundary node on a
// Dirichlet face, are decoupled.  The generalised eigenproblem A s = lambda B s
// (eq. 6) of the coupled block is solved with B diagonal: cyclic Jacobi on
// B^{-1/2} A B^{-1/2} = V Lambda V^T, S = B^{-1/2} V, so S^T A S = Lambda and
// S^T B S = I (eq. 7).  Decoupled nodes get identity columns and lambda = +inf.
//
// Apply (eq. 8): gather the (p+3)^3 box from the consistent E-vector (overlap
// values come from face, edge and corner neighbours; outside the domain 0),
// contract with S_x^T, S_y^T, S_z^T, divide by lambda_x + lambda_y + lambda_z
// (eq. 9), contract back with S, and keep the element's own (p+1)^3 nodes
// times the RAS weight 1/multiplicity; the caller then assembles (QQ^T).
#include "sem_internal.h"

namespace sem {

constexpr int kMaxPB = kMaxP + 3;

__global__ __launch_bounds__(64) void k_fdm_setup(int64_t E, int p, int nex, int ney, int nez,
                                                  int bc0, int bc1, int bc2, int bc3, int bc4,
                                                  int bc5, const double *__restrict__ D,
                                                  const double *__restrict__ wq,
                                                  const double *__restrict__ boxlen,
                                                  double *__restrict__ S64,
                                                  double *__restrict__ lam64,
                                                  float *__restrict__ S32,
                                                  float *__restrict__ lam32) {
  const int N = p + 1, pb = p + 3;
  __shared__ double Ah[(kMaxP + 1) * (kMaxP + 1)];
  __shared__ double ws[kMaxP + 1];
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
    int a = t / N, b = t % N;
    double s = 0;
    for (int q = 0; q < N; ++q) s += D[q * N + a] * wq[q] * D[q * N + b];
    Ah[t] = s;
  }
  for (int t = threadIdx.x; t < N; t += blockDim.x) ws[t] = wq[t];
  __syncthreads();

  int64_t task = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (task >= 3 * E) return;
  const int64_t e = task / 3;
  const int d = (int)(task - e * 3);
  const int64_t ex = e % nex, ey = (e / nex) % ney, ez = e / ((int64_t)nex * ney);
  const int64_t pos = d == 0 ? ex : d == 1 ? ey : ez;
  const int64_t cnt = d == 0 ? nex : d == 1 ? ney : nez;
  const int64_t stride = d == 0 ? 1 : d == 1 ? nex : (int64_t)nex * ney;
  const bool has_l = pos > 0, has_r = pos < cnt - 1;
  const int dir_l = d == 0 ? bc0 : d == 1 ? bc2 : bc4;
  const int dir_r = d == 0 ? bc1 : d == 1 ? bc3 : bc5;
  const double Lc = boxlen[e * 3 + d];
  const double Lm = has_l ? boxlen[(e - stride) * 3 + d] : 0.0;
  const double Lp = has_r ? boxlen[(e + stride) * 3 + d] : 0.0;

  // extended node q sits at chain index c = p - 1 + q of the 3-element chain
  double K[kMaxPB * kMaxPB], M[kMaxPB];
  for (int q1 = 0; q1 < pb; ++q1) {
    M[q1] = 0.0;
    for (int q2 = 0; q2 < pb; ++q2) K[q1 * kMaxPB + q2] = 0.0;
  }
  for (int t = 0; t < 3; ++t) {
    bool present = t == 1 || (t == 0 && has_l) || (t == 2 && has_r);
    if (!present) continue;
    double Le = t == 0 ? Lm : t == 1 ? Lc : Lp;
    for (int q1 = 0; q1 < pb; ++q1) {
      int a = p - 1 + q1 - t * p;
      if (a < 0 || a > p) continue;
      M[q1] += 0.5 * Le * ws[a];
      for (int q2 = 0; q2 < pb; ++q2) {
        int b = p - 1 + q2 - t * p;
        if (b < 0 || b > p) continue;
        K[q1 * kMaxPB + q2] += (2.0 / Le) * Ah[a * N + b];
      }
    }
  }
  bool cpl[kMaxPB];
  for (int q = 0; q < pb; ++q) cpl[q] = true;
  if (!has_l) {
    cpl[0] = false;
    if (dir_l) cpl[1] = false;
  }
  if (!has_r) {
    cpl[pb - 1] = false;
    if (dir_r) cpl[pb - 2] = false;
  }
  int idx[kMaxPB], m = 0;
  for (int q = 0; q < pb; ++q)
    if (cpl[q]) idx[m++] = q;

  // C = M^{-1/2} K M^{-1/2} on the coupled nodes; cyclic Jacobi C = V Lambda V^T
  double C[kMaxPB * kMaxPB], V[kMaxPB * kMaxPB], mh[kMaxPB];
  for (int a = 0; a < m; ++a) mh[a] = 1.0 / sqrt(M[idx[a]]);
  double fro = 0.0;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      double v = mh[a] * K[idx[a] * kMaxPB + idx[b]] * mh[b];
      C[a * kMaxPB + b] = v;
      V[a * kMaxPB + b] = (a == b) ? 1.0 : 0.0;
      fro += v * v;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int a = 0; a < m; ++a)
      for (int b = a + 1; b < m; ++b) off += C[a * kMaxPB + b] * C[a * kMaxPB + b];
    if (off <= 1e-32 * fro) break;
    for (int a = 0; a < m; ++a)
      for (int b = a + 1; b < m; ++b) {
        double apq = C[a * kMaxPB + b];
        if (fabs(apq) < 1e-300) continue;
        double theta = (C[b * kMaxPB + b] - C[a * kMaxPB + a]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {  // columns a, b
          double ka = C[k * kMaxPB + a], kb = C[k * kMaxPB + b];
          C[k * kMaxPB + a] = c * ka - s * kb;
          C[k * kMaxPB + b] = s * ka + c * kb;
        }
        for (int k = 0; k < m; ++k) {  // rows a, b
          double ak = C[a * kMaxPB + k], bk = C[b * kMaxPB + k];
          C[a * kMaxPB + k] = c * ak - s * bk;
          C[b * kMaxPB + k] = s * ak + c * bk;
        }
        C[a * kMaxPB + b] = 0.0;
        C[b * kMaxPB + a] = 0.0;
        for (int k = 0; k < m; ++k) {
          double va = V[k * kMaxPB + a], vb = V[k * kMaxPB + b];
          V[k * kMaxPB + a] = c * va - s * vb;
          V[k * kMaxPB + b] = s * va + c * vb;
        }
      }
  }
  double lmax = 0.0;
  for (int a = 0; a < m; ++a) lmax = fmax(lmax, fabs(C[a * kMaxPB + a]));

  // S[q][col] (row = extended node, column = mode), lambda[col]
  double *Se = S64 + (e * 3 + d) * pb * pb;
  double *le = lam64 + (e * 3 + d) * pb;
  for (int q = 0; q < pb; ++q)
    for (int a = 0; a < pb; ++a) Se[q * pb + a] = 0.0;
  for (int a = 0; a < m; ++a) {
    double lv = C[a * kMaxPB + a];
    le[a] = fabs(lv) <= 1e-12 * lmax ? 0.0 : lv;
    for (int r = 0; r < m; ++r) Se[idx[r] * pb + a] = mh[r] * V[r * kMaxPB + a];
  }
  int col = m;
  for (int q = 0; q < pb; ++q)
    if (!cpl[q]) {
      Se[q * pb + col] = 1.0;
      le[col] = __builtin_huge_val();
      ++col;
    }
  if (S32) {
    float *Sf = S32 + (e * 3 + d) * pb * pb;
    float *lf = lam32 + (e * 3 + d) * pb;
    for (int q = 0; q < pb * pb; ++q) Sf[q] = (float)Se[q];
    for (int a = 0; a < pb; ++a) lf[a] = (float)le[a];
  }
}

void launch_fdm_setup(const Ctx &c, Level &L, hipStream_t s) {
  int64_t tasks = 3 * L.E;
  hipLaunchKernelGGL(k_fdm_setup, dim3((unsigned)((tasks + 63) / 64)), dim3(64), 0, s, L.E, L.p,
                     c.nex, c.ney, c.nez, c.bc[0], c.bc[1], c.bc[2], c.bc[3], c.bc[4], c.bc[5],
                     L.D64, L.wq, L.boxlen, L.S64, L.lam64, L.S32, L.lam32);
  SEM_LAUNCH("k_fdm_setup");
}

// ---------------------------------------------------------------------------
// apply: one element per workgroup, thread (a, b) owns the box column
// (a, b, 0..pb-1) in registers; the x and y contractions go through LDS.
// Boxes with fewer than 64 lines (p <= 4) can put EB elements in one workgroup
// of at most TMAX threads so that the lanes of its wavefronts are nearly all
// busy (36 lines per element at p = 3 leave 28 of 64 lanes idle; 7 elements fill
// 252 of 256 lanes).  EB is the count within TMAX threads and 32 KB of LDS with
// the best lane use.  Measured on the p = 3 level of a 32^3 mesh: 256 threads
// beat one wavefront by 10 % (FP32) and 1024 threads (fewer workgroups in
// flight between barriers); at p = 4 one wavefront per element stays faster.
constexpr int fdm_group(int pb2, int lim) {
  int best = 1;
  for (int e = 2; e <= lim; ++e) {
    const long ue = (long)e * pb2 * (((best * pb2 + 63) / 64) * 64);
    const long ub = (long)best * pb2 * (((e * pb2 + 63) / 64) * 64);
    if (ue > ub) best = e;
  }
  return best;
}
template <int P, typename T, int TMAX>
struct FdmShape {
  static constexpr int PB = P + 3;
  static constexpr int N = P + 1;
  static constexpr int PB2 = PB * PB;
  static constexpr int RS = PB;
  static constexpr int PS = PB * RS;
  static constexpr int EB_T = TMAX / PB2;
  static constexpr int EB_L = 32768 / (2 * PB * PS * (int)sizeof(T));
  static constexpr int EB = PB2 >= 64 ? 1 : fdm_group(PB2, EB_T < EB_L ? EB_T : EB_L);
  static constexpr int BS = ((EB * PB2 + 63) / 64) * 64;
};

template <typename T>
__device__ inline T fdm_inv(T d) {
  return d > T(0) ? T(1) / d : T(0);  // +inf -> 0 (decoupled), 0 -> dropped mode
}
// FP32: the hardware reciprocal (about 1 ulp) instead of the IEEE division
template <>
__device__ inline float fdm_inv<float>(float d) {
  return d > 0.f ? __builtin_amdgcn_rcpf(d) : 0.f;
}

// rs (may be null): the local solves act on r - rs (a residual formed as read)
template <int P, typename T, bool ASM, int TMAX>
__global__ __launch_bounds__((FdmShape<P, T, TMAX>::BS)) void k_fdm(
    int64_t E, int nex, int ney, int nez, const T *__restrict__ r, const T *__restrict__ rs,
    const T *__restrict__ Sg, const T *__restrict__ lamg, const T *__restrict__ W,
    T *__restrict__ z, int nv) {
  using F = FdmShape<P, T, TMAX>;
  constexpr int PB = F::PB, N = F::N, RS = F::RS, PS = F::PS, EB = F::EB;
  constexpr int N3 = N * N * N, PB2 = PB * PB;
  __shared__ T sb0[EB][PB * PS];
  __shared__ T sb1[EB][PB * PS];
  __shared__ T sZ[EB][EB > 1 ? PB2 + PB : 1];  // S_z, lambda_z of each element of a group

  int vec;
  const int64_t grp = split_rhs(xcd_block(), nv, vec);
  r += (int64_t)vec * E * N3;
  if (rs) rs += (int64_t)vec * E * N3;
  z += (int64_t)vec * E * N3;
  const int tid = threadIdx.x;
  // element of the group (0 when the group is one element: e stays uniform)
  const int lel = EB == 1 ? 0 : tid / PB2, lt = tid - lel * PB2;
  const int a = lt % PB, b = lt / PB;
  const int64_t e = (int64_t)grp * EB + lel;
  const bool act = (EB == 1 ? tid < PB2 : lel < EB) && e < E;
  T *buf0 = sb0[lel < EB ? lel : 0];
  T *buf1 = sb1[lel < EB ? lel : 0];
  // the thread's rows and columns of S_x (index a) and S_y (index b) live in
  // registers; S_z and lambda_z are the same for the element's lanes (scalar
  // loads when the workgroup holds one element, else staged in LDS)
  const int64_t es = e < E ? e : E - 1;  // uniform when the group is one element
  const T *Se = Sg + es * 3 * PB2;
  const T *le = lamg + es * 3 * PB;
  const T *__restrict__ Sz = Se + 2 * PB2;
  const T *__restrict__ lz = le + 2 * PB;
  T Sxc[PB], Sxr[PB], Syc[PB], Syr[PB];
  T lxy = T(0);
  if (act) {
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      Sxc[q] = Se[q * PB + a];
      Sxr[q] = Se[a * PB + q];
      Syc[q] = Se[PB2 + q * PB + b];
      Syr[q] = Se[PB2 + b * PB + q];
    }
    lxy = le[a] + le[PB + b];
  }

  int64_t ex, ey, ez;
  elem_coords(e, nex, ney, ex, ey, ez);
  T col[PB];
  if (act) {
    // box node (a, b, c): direction offsets and local indices; one base pointer
    // per column, unconditional loads, as in k_fdm_lines
    const int dx = a == 0 ? -1 : (a == PB - 1 ? 1 : 0);
    const int li = a == 0 ? P - 1 : (a == PB - 1 ? 1 : a - 1);
    const int dy = b == 0 ? -1 : (b == PB - 1 ? 1 : 0);
    const int lj = b == 0 ? P - 1 : (b == PB - 1 ? 1 : b - 1);
    const bool okxy = (ex + dx >= 0) && (ex + dx < nex) && (ey + dy >= 0) && (ey + dy < ney);
    const bool okd = okxy && ez > 0, oku = okxy && ez + 1 < nez;
    const int64_t plane = (int64_t)nex * ney * N3;
    const int64_t base = (okxy ? e + dx + (int64_t)dy * nex : e) * N3 + lj * N + li;
    const T *cp = r + base;
    const int64_t od = okd ? (P - 1) * N * N - plane : 0, ou = oku ? N * N + plane : 0;
    T lower = cp[od];
    T upper = cp[ou];
#pragma unroll
    for (int c = 1; c < PB - 1; ++c) col[c] = cp[(c - 1) * N * N];
    if (rs) {
      const T *cs = rs + base;
      lower -= cs[od];
      upper -= cs[ou];
#pragma unroll
      for (int c = 1; c < PB - 1; ++c) col[c] -= cs[(c - 1) * N * N];
    }
#pragma unroll
    for (int c = 1; c < PB - 1; ++c) col[c] = okxy ? col[c] : T(0);
    col[0] = okd ? lower : T(0);
    col[PB - 1] = oku ? upper : T(0);
#pragma unroll
    for (int c = 0; c < PB; ++c) buf0[c * PS + b * RS + a] = col[c];
    if constexpr (EB > 1) {
      sZ[lel][lt] = Sz[lt];
      if (lt < PB) sZ[lel][PB2 + lt] = lz[lt];
    }
  }
  __syncthreads();
  // x: t[c][b][a] = sum_i Sx[i][a] box[c][b][i]
  if (act) {
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      T s = 0;
#pragma unroll
      for (int i = 0; i < PB; ++i) s += Sxc[i] * buf0[c * PS + b * RS + i];
      buf1[c * PS + b * RS + a] = s;
    }
  }
  __syncthreads();
  // y: t[c][b][a] = sum_j Sy[j][b] t[c][j][a]; then z in registers
  if (act) {
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < PB; ++j) s += Syc[j] * buf1[c * PS + j * RS + a];
      col[c] = s;
    }
    // along z and back: S_z from scalar loads (one element) or LDS (a group)
    auto zpass = [&](const T *SZ, const T *LZ) {
      T h[PB];
#pragma unroll
      for (int cc = 0; cc < PB; ++cc) {
        T s = 0;
#pragma unroll
        for (int k = 0; k < PB; ++k) s += SZ[k * PB + cc] * col[k];
        h[cc] = s * fdm_inv<T>(lxy + LZ[cc]);
      }
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        T s = 0;
#pragma unroll
        for (int cc = 0; cc < PB; ++cc) s += SZ[k * PB + cc] * h[cc];
        col[k] = s;
      }
    };
    if constexpr (EB > 1)
      zpass(sZ[lel], sZ[lel] + PB2);
    else
      zpass(Sz, lz);
#pragma unroll
    for (int c = 0; c < PB; ++c) buf0[c * PS + b * RS + a] = col[c];
  }
  __syncthreads();
  // back along y: y[c][j][a] = sum_bb Sy[j][bb] t[c][bb][a]   (thread (a, j = b))
  if (act) {
#pragma unroll
    for (int c = 0; c < PB; ++c) {
      T s = 0;
#pragma unroll
      for (int bb = 0; bb < PB; ++bb) s += Syr[bb] * buf0[c * PS + bb * RS + a];
      buf1[c * PS + b * RS + a] = s;
    }
  }
  __syncthreads();
  // back along x: out[c][j][i] = sum_aa Sx[i][aa] y[c][j][aa]
  if constexpr (ASM) {  // whole box to z[E][pb^3]; the overlap sum follows
    if (act) {
      T *zb = z + e * PB * PB * PB + b * PB + a;
#pragma unroll
      for (int c = 0; c < PB; ++c) {
        T s = 0;
#pragma unroll
        for (int aa = 0; aa < PB; ++aa) s += Sxr[aa] * buf1[c * PS + b * RS + aa];
        zb[c * PB * PB] = s;
      }
    }
    return;
  }
  // RAS output on own nodes, times 1/multiplicity
  if (act && a >= 1 && a <= P + 1 && b >= 1 && b <= P + 1) {
    const int64_t obase = e * N3 + (b - 1) * N + (a - 1);
#pragma unroll
    for (int c = 1; c <= P + 1; ++c) {
      T s = 0;
#pragma unroll
      for (int aa = 0; aa < PB; ++aa) s += Sxr[aa] * buf1[c * PS + b * RS + aa];
      const int64_t o = obase + (int64_t)(c - 1) * N * N;
      z[o] = W[o] * s;
    }
  }
}

// Same local solve, organised by lines: in each contraction a thread owns one
// line of the box along the contracted direction, reads its pbar values from
// LDS once and forms all pbar outputs, with the entries of S taken as
// block-uniform (scalar-loaded) operands.  That is one LDS read per pbar
// multiply-adds instead of one per multiply-add.  The RAS write-out has the
// thread (b, c) own the row of pbar-2 = p+1 consecutive output values, so the
// element's (p+1)^3 outputs leave as contiguous rows.  Used for pbar^2 > 64.
template <int P>
struct FdmLines {
  static constexpr int PB = P + 3;
  static constexpr int N = P + 1;
  static constexpr int BS = ((PB * PB + 63) / 64) * 64;
  static constexpr int RS = PB | 1;
  static constexpr int PS = PB * RS;  // fewer bank conflicts than an odd plane stride (modelled)
};

template <int P, typename T, bool ASM>
__global__ __launch_bounds__(FdmLines<P>::BS) void k_fdm_lines(
    int64_t E, int nex, int ney, int nez, const T *__restrict__ r, const T *__restrict__ rs,
    const T *__restrict__ Sg, const T *__restrict__ lamg, const T *__restrict__ W,
    T *__restrict__ z, int nv) {
  using F = FdmLines<P>;
  constexpr int PB = F::PB, N = F::N, RS = F::RS, PS = F::PS;
  constexpr int N3 = N * N * N, PB2 = PB * PB;
  __shared__ T buf0[PB * PS];
  __shared__ T buf1[PB * PS];

  int vec;
  const int64_t e = split_rhs(xcd_block(), nv, vec);
  r += (int64_t)vec * E * N3;
  if (rs) rs += (int64_t)vec * E * N3;
  z += (int64_t)vec * E * N3;
  const int tid = threadIdx.x;
  const bool act = tid < PB2;
  const int lo = tid % PB, hi = tid / PB;  // the two free box indices of this thread's line
  const T *__restrict__ Sx = Sg + e * 3 * PB2;
  const T *__restrict__ Sy = Sx + PB2;
  const T *__restrict__ Sz = Sx + 2 * PB2;
  const T *__restrict__ le = lamg + e * 3 * PB;
  T v[PB], o[PB];

  // gather the box: thread (a, b) = (lo, hi) reads the line along c.  One base
  // pointer per line (the x/y neighbour's column) and compile-time offsets for
  // the planes; the two overlap planes come from the z neighbours.  Loads are
  // unconditional (an outside neighbour reads the element itself and is
  // replaced by 0), so that all PB loads are in flight together.
  {
    int64_t ex, ey, ez;
    elem_coords(e, nex, ney, ex, ey, ez);
    if (act) {
      const int a = lo, b = hi;
      const int dx = a == 0 ? -1 : (a == PB - 1 ? 1 : 0);
      const int li = a == 0 ? P - 1 : (a == PB - 1 ? 1 : a - 1);
      const int dy = b == 0 ? -1 : (b == PB - 1 ? 1 : 0);
      const int lj = b == 0 ? P - 1 : (b == PB - 1 ? 1 : b - 1);
      const bool okxy = (ex + dx >= 0) && (ex + dx < nex) && (ey + dy >= 0) && (ey + dy < ney);
      const bool okd = okxy && ez > 0, oku = okxy && ez + 1 < nez;
      const int64_t plane = (int64_t)nex * ney * N3;
      const int64_t base = (okxy ? e + dx + (int64_t)dy * nex : e) * N3 + lj * N + li;
      const T *col = r + base;
      const int64_t od = okd ? (P - 1) * N * N - plane : 0, ou = oku ? N * N + plane : 0;
      T lower = col[od];
      T upper = col[ou];
#pragma unroll
      for (int c = 1; c < PB - 1; ++c) v[c] = col[(c - 1) * N * N];
      if (rs) {  // r - rs: the residual formed as it is read
        const T *cs = rs + base;
        lower -= cs[od];
        upper -= cs[ou];
#pragma unroll
        for (int c = 1; c < PB - 1; ++c) v[c] -= cs[(c - 1) * N * N];
      }
#pragma unroll
      for (int c = 1; c < PB - 1; ++c) v[c] = okxy ? v[c] : T(0);
      v[0] = okd ? lower : T(0);
      v[PB - 1] = oku ? upper : T(0);
#pragma unroll
      for (int c = 0; c < PB; ++c) buf0[c * PS + b * RS + a] = v[c];
    }
  }
  __syncthreads();
  // x: t[c][b][m] = sum_i Sx[i][m] box[c][b][i]      line (b, c) = (lo, hi)
  if (act) {
    const int b = lo, c = hi;
#pragma unroll
    for (int i = 0; i < PB; ++i) v[i] = buf0[c * PS + b * RS + i];
#pragma unroll
    for (int m = 0; m < PB; ++m) o[m] = T(0);
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int m = 0; m < PB; ++m) o[m] += Sx[i * PB + m] * v[i];
#pragma unroll
    for (int m = 0; m < PB; ++m) buf1[c * PS + b * RS + m] = o[m];
  }
  __syncthreads();
  // y: t[c][m][a] = sum_j Sy[j][m] t[c][j][a]         line (a, c) = (lo, hi)
  if (act) {
    const int a = lo, c = hi;
#pragma unroll
    for (int j = 0; j < PB; ++j) v[j] = buf1[c * PS + j * RS + a];
#pragma unroll
    for (int m = 0; m < PB; ++m) o[m] = T(0);
#pragma unroll
    for (int j = 0; j < PB; ++j)
#pragma unroll
      for (int m = 0; m < PB; ++m) o[m] += Sy[j * PB + m] * v[j];
#pragma unroll
    for (int m = 0; m < PB; ++m) buf0[c * PS + m * RS + a] = o[m];
  }
  __syncthreads();
  // z forward, divide by lambda_x + lambda_y + lambda_z, z back   line (a, b)
  if (act) {
    const int a = lo, b = hi;
    const T lxy = le[a] + le[PB + b];
#pragma unroll
    for (int k = 0; k < PB; ++k) v[k] = buf0[k * PS + b * RS + a];
#pragma unroll
    for (int m = 0; m < PB; ++m) o[m] = T(0);
#pragma unroll
    for (int k = 0; k < PB; ++k)
#pragma unroll
      for (int m = 0; m < PB; ++m) o[m] += Sz[k * PB + m] * v[k];
#pragma unroll
    for (int m = 0; m < PB; ++m) o[m] *= fdm_inv<T>(lxy + le[2 * PB + m]);
    // RAS keeps the element's own nodes only: the way back needs planes
    // k = 1..p+1 (and below, rows j = 1..p+1); ASM needs the whole box
    constexpr int K0 = ASM ? 0 : 1, K1 = ASM ? PB : PB - 1;
#pragma unroll
    for (int k = K0; k < K1; ++k) v[k] = T(0);
#pragma unroll
    for (int m = 0; m < PB; ++m)
#pragma unroll
      for (int k = K0; k < K1; ++k) v[k] += Sz[k * PB + m] * o[m];
#pragma unroll
    for (int k = K0; k < K1; ++k) buf1[k * PS + b * RS + a] = v[k];
  }
  __syncthreads();
  // y back: t[c][j][a] = sum_m Sy[j][m] t[c][m][a]    line (a, c)
  if (act && (ASM || (hi >= 1 && hi <= PB - 2))) {
    constexpr int J0 = ASM ? 0 : 1, J1 = ASM ? PB : PB - 1;
    const int a = lo, c = hi;
#pragma unroll
    for (int m = 0; m < PB; ++m) v[m] = buf1[c * PS + m * RS + a];
#pragma unroll
    for (int j = J0; j < J1; ++j) o[j] = T(0);
#pragma unroll
    for (int m = 0; m < PB; ++m)
#pragma unroll
      for (int j = J0; j < J1; ++j) o[j] += Sy[j * PB + m] * v[m];
#pragma unroll
    for (int j = J0; j < J1; ++j) buf0[c * PS + j * RS + a] = o[j];
  }
  __syncthreads();
  // x back: out[c][b][i] = sum_m Sx[i][m] t[c][b][m]
  if constexpr (ASM) {  // whole box to z[E][pb^3]; the overlap sum follows
    if (act) {
      const int b = lo, c = hi;
#pragma unroll
      for (int m = 0; m < PB; ++m) v[m] = buf0[c * PS + b * RS + m];
#pragma unroll
      for (int i = 0; i < PB; ++i) o[i] = T(0);
#pragma unroll
      for (int m = 0; m < PB; ++m)
#pragma unroll
        for (int i = 0; i < PB; ++i) o[i] += Sx[i * PB + m] * v[m];
      T *zb = z + e * PB * PB2 + c * PB2 + b * PB;
#pragma unroll
      for (int i = 0; i < PB; ++i) zb[i] = o[i];
    }
    return;
  }
  // RAS: own rows (b, c) in 1..p+1, outputs i in 1..p+1, times 1/multiplicity
  if (tid < N * N) {
    const int b = 1 + tid % N, c = 1 + tid / N;
#pragma unroll
    for (int m = 0; m < PB; ++m) v[m] = buf0[c * PS + b * RS + m];
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = T(0);
#pragma unroll
    for (int m = 0; m < PB; ++m)
#pragma unroll
      for (int i = 0; i < N; ++i) o[i] += Sx[(i + 1) * PB + m] * v[m];
    const int64_t row = e * N3 + (int64_t)(c - 1) * N * N + (b - 1) * N;
#pragma unroll
    for (int i = 0; i < N; ++i) z[row + i] = W[row + i] * o[i];
  }
}

// ASM (eq. 4): sum of every extended box that contains the node, times
// 1/#boxes, masked.  Each local copy of a node sums the same boxes, so the
// result is a consistent E-vector without a separate assembly.
template <typename T>
__global__ void k_asm_sum(int64_t E, int p, int nex, int ney, int nez, const T *__restrict__ box,
                          const T *__restrict__ w, T *__restrict__ z) {
  const int N = p + 1, N3 = N * N * N, PB = p + 3, PB3 = PB * PB * PB;
  int64_t t = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  if (t >= E * N3) return;
  if (w[t] == T(0)) {  // Dirichlet node
    z[t] = T(0);
    return;
  }
  int64_t e = t / N3;
  int q = (int)(t - e * N3);
  int i = q % N, j = (q / N) % N, k = q / (N * N);
  int64_t ex = e % nex, ey = (e / nex) % ney, ez = e / ((int64_t)nex * ney);
  int64_t gx = ex * p + i, gy = ey * p + j, gz = ez * p + k;
  T sum = T(0);
  int cnt = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    int64_t cz = ez + dz;
    int64_t lz = gz - cz * p + 1;
    if (cz < 0 || cz >= nez || lz < 0 || lz >= PB) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int64_t cy = ey + dy;
      int64_t ly = gy - cy * p + 1;
      if (cy < 0 || cy >= ney || ly < 0 || ly >= PB) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        int64_t cx = ex + dx;
        int64_t lx = gx - cx * p + 1;
        if (cx < 0 || cx >= nex || lx < 0 || lx >= PB) continue;
        int64_t en = (cz * ney + cy) * nex + cx;
        sum += box[en * PB3 + (lz * PB + ly) * PB + lx];
        ++cnt;
      }
    }
  }
  z[t] = sum / T(cnt);
}

template <typename T>
void launch_asm_sum(const Ctx &c, const Level &L, const T *box, T *z, hipStream_t s) {
  const T *w = sizeof(T) == 8 ? (const T *)L.w64 : (const T *)L.w32;
  hipLaunchKernelGGL(k_asm_sum<T>, dim3((unsigned)((L.nloc + 255) / 256)), dim3(256), 0, s, L.E,
                     L.p, c.nex, c.ney, c.nez, box, w, z);
  SEM_LAUNCH("k_asm_sum");
}
template void launch_asm_sum<double>(const Ctx &, const Level &, const double *, double *,
                                     hipStream_t);
template void launch_asm_sum<float>(const Ctx &, const Level &, const float *, float *,
                                    hipStream_t);

template <int P, typename T, bool ASM, int TMAX>
static void fdm_launch_grouped(const Ctx &c, const Level &L, const T *r, const T *rs, const T *S,
                               const T *lam, const T *W, T *out, hipStream_t s, int nv) {
  using F = FdmShape<P, T, TMAX>;
  const dim3 grid((unsigned)((L.E + F::EB - 1) / F::EB * nv));
  hipLaunchKernelGGL((k_fdm<P, T, ASM, TMAX>), grid, dim3(F::BS), 0, s, L.E, c.nex, c.ney, c.nez,
                     r, rs, S, lam, W, out, nv);
}

template <int P, typename T, bool ASM>
static void fdm_launch(const Ctx &c, const Level &L, const T *r, const T *rs, const T *S,
                       const T *lam, const T *W, T *out, hipStream_t s, int nv) {
  const dim3 grid((unsigned)(L.E * nv));
  if (FdmLines<P>::PB * FdmLines<P>::PB > 64 && c.fdm_lines)
    hipLaunchKernelGGL((k_fdm_lines<P, T, ASM>), grid, dim3(FdmLines<P>::BS), 0, s, L.E, c.nex,
                       c.ney, c.nez, r, rs, S, lam, W, out, nv);
  else if (P <= 3 && c.fdm_group)  // measured: faster up to p = 3, slower at p = 4
    fdm_launch_grouped<P, T, ASM, (P <= 3 ? 256 : 64)>(c, L, r, rs, S, lam, W, out, s, nv);
  else
    fdm_launch_grouped<P, T, ASM, 64>(c, L, r, rs, S, lam, W, out, s, nv);
  SEM_LAUNCH("k_fdm");
}

template <typename T, int P>
static void fdm_p(const Ctx &c, const Level &L, const T *r, T *z, bool asm_mode, hipStream_t s,
                  int nv, const T *rs, int xin) {
  const T *S = sizeof(T) == 8 ? (const T *)L.S64 : (const T *)L.S32;
  const T *lam = sizeof(T) == 8 ? (const T *)L.lam64 : (const T *)L.lam32;
  const T *W = sizeof(T) == 8 ? (const T *)L.w64 : (const T *)L.w32;
  if (!S || !lam || !W) fail(SEM_EINVAL, "FDM data of this precision were not built");
  if (asm_mode) {
    T *box = sizeof(T) == 8 ? (T *)L.box64 : (T *)L.box32;
    if (!box) fail(SEM_EINVAL, "ASM box buffer was not built");
    for (int k = 0; k < nv; ++k) {  // one box buffer: right sides in turn
      fdm_launch<P, T, true>(c, L, r + k * L.nloc, rs ? rs + k * L.nloc : nullptr, S, lam, W, box,
                             s, 1);
      launch_asm_sum<T>(c, L, box, z + k * L.nloc, s);
    }
    return;
  }
  if constexpr (sizeof(T) == 4) {
    if (c.fdm_mf32 && fdm_mf32_supported(c, P)) {
      launch_fdm_mf32(c, L, (const float *)r, (float *)z, s, nv, (const float *)rs, xin);
      return;
    }
  }
  if (xin) fail(SEM_EINVAL, "FDM: this kernel needs assembled inputs");
  fdm_launch<P, T, false>(c, L, r, rs, S, lam, W, z, s, nv);
}

template <typename T>
void launch_fdm(const Ctx &c, const Level &L, const T *r, T *z, bool asm_mode, hipStream_t s,
                int nv, const T *rs, int xin) {
  if (xin && asm_mode) fail(SEM_EINVAL, "FDM: ASM needs assembled inputs");
  switch (L.p) {
    case 2: fdm_p<T, 2>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 3: fdm_p<T, 3>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 4: fdm_p<T, 4>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 5: fdm_p<T, 5>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 6: fdm_p<T, 6>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 7: fdm_p<T, 7>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 8: fdm_p<T, 8>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 9: fdm_p<T, 9>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    case 10: fdm_p<T, 10>(c, L, r, z, asm_mode, s, nv, rs, xin); break;
    default: fail(SEM_EUNSUPPORTED, "FDM: unsupported degree");
  }
}
template void launch_fdm<double>(const Ctx &, const Level &, const double *, double *, bool,
                                 hipStream_t, int, const double *, int);
template void launch_fdm<float>(const Ctx &, const Level &, const float *, float *, bool,
                                hipStream_t, int, const float *, int);

}  // namespace sem
