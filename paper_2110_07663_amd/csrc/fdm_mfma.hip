// FDM local solves (Sec. 2.2.2, eqs. 8-9) with the six 1D contractions on the
// matrix cores: BF16 or FP16 operands, FP32 accumulation.
//
// Each contraction of the (p+3)^3 box with a (p+3)x(p+3) factor is one GEMM
// whose rows are the pairs of the two untouched indices (pbar^2 <= 169 rows,
// tiles of 16) and whose inner dimension is the contracted index (pbar <= 16,
// zero-padded): D[m][n] = sum_k A[m][k] B[k][n] with v_mfma_f32_16x16x16
// (one wave per element).  Operand fragments (64 lanes):
//   A: lane l holds A[l % 16][4 (l / 16) + j], j < 4
//   B: lane l holds B[4 (l / 16) + j][l % 16]
//   D: lane l holds D[4 (l / 16) + j][l % 16]
// The box stays in LDS in FP32 between contractions.  Narrow formats need
// bounded magnitudes, so every element's box is divided by its largest entry
// before the forward pass, the factors S_d are stored divided by their largest
// entry s_d (in [-1, 1]), and the diagonally scaled tensor is renormalised
// before the backward pass; the scalars are restored on output.
#include "sem_internal.h"

namespace sem {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline uint16_t f32_to_f16_bits(float x) {
  _Float16 h = (_Float16)x;
  return *reinterpret_cast<uint16_t *>(&h);
}

template <bool BF>
struct Mma;
template <>
struct Mma<true> {  // BF16
  using frag = short4_t;
  static __device__ inline short enc(float x) { return (short)f32_to_bf16_rne(x); }
  static __device__ inline short from_bits(uint16_t b) { return (short)b; }
  static __device__ inline float4_t mma(frag a, frag b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<false> {  // FP16
  using frag = half4_t;
  static __device__ inline _Float16 enc(float x) { return (_Float16)x; }
  static __device__ inline _Float16 from_bits(uint16_t b) {
    return *reinterpret_cast<_Float16 *>(&b);
  }
  static __device__ inline float4_t mma(frag a, frag b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

__device__ inline float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// setup: S16[e][d][q][a] = S[e][d][q][a] / s_d (16-bit pattern), sscale[e][d] = s_d
__global__ void k_fdm_pack16(int64_t E, int pb, const float *__restrict__ S32,
                             uint16_t *__restrict__ S16, float *__restrict__ sscale, int bf) {
  int64_t task = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (task >= 3 * E) return;
  const float *Sd = S32 + task * pb * pb;
  float m = 0.f;
  for (int q = 0; q < pb * pb; ++q) m = fmaxf(m, fabsf(Sd[q]));
  float inv = m > 0.f ? 1.f / m : 0.f;
  uint16_t *o = S16 + task * pb * pb;
  for (int q = 0; q < pb * pb; ++q) {
    float v = Sd[q] * inv;
    o[q] = bf ? f32_to_bf16_rne(v) : f32_to_f16_bits(v);
  }
  sscale[task] = m;
}

// Operand view of the box in LDS for a contraction along direction `dir`:
// rows m = (u, v) pairs of the other two indices, k = contracted index.
template <int PB, int RS, int PS>
__device__ inline int box_index(int dir, int m, int k) {
  int hi = m / PB, lo = m - hi * PB;
  // dir 0 (x): m = (c, b), k = a;  dir 1 (y): m = (c, a), k = b;  dir 2 (z): m = (b, a), k = c
  if (dir == 0) return hi * PS + lo * RS + k;
  if (dir == 1) return hi * PS + k * RS + lo;
  return k * PS + hi * RS + lo;
}

template <int P, bool BF, bool ASM>
__global__ __launch_bounds__(256) void k_fdm_mfma(int64_t E, int nex, int ney, int nez,
                                                  const float *__restrict__ r,
                                                  const uint16_t *__restrict__ S16,
                                                  const float *__restrict__ sscale,
                                                  const float *__restrict__ lam,
                                                  const float *__restrict__ W,
                                                  float *__restrict__ z, int nv) {
  using M = Mma<BF>;
  using frag = typename M::frag;
  constexpr int PB = P + 3, N = P + 1, N3 = N * N * N;
  constexpr int RS = PB + 1, PS = PB * RS, BOX = PB * PS;
  constexpr int MROWS = PB * PB;
  constexpr int TILES = (MROWS + 15) / 16;
  constexpr int WAVES = 4;
  static_assert(PB <= 16, "pbar must fit one 16-wide tile");
  __shared__ float buf[WAVES][2][BOX];
  __shared__ float sl[WAVES][3][PB];

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  int vec;
  const int64_t e = (int64_t)split_rhs(xcd_block(), nv, vec) * WAVES + wave;
  if (e >= E) return;  // whole wave leaves; no block-wide barriers below
  r += (int64_t)vec * E * N3;  // right side vec (RAS: output E-vectors nloc apart)
  z += (int64_t)vec * E * N3;
  float *X = buf[wave][0];
  float *Y = buf[wave][1];

  // B fragments: forward B[k][n] = Shat_d[k][n], backward B[k][n] = Shat_d[n][k]
  const int col = lane % 16, kb = 4 * (lane / 16);
  frag Bf[3], Bb[3];
  const uint16_t *Se = S16 + e * 3 * PB * PB;
  for (int d = 0; d < 3; ++d) {
    for (int j = 0; j < 4; ++j) {
      int k = kb + j;
      bool ok = k < PB && col < PB;
      uint16_t f = ok ? Se[(d * PB + k) * PB + col] : (uint16_t)0;
      uint16_t b = ok ? Se[(d * PB + col) * PB + k] : (uint16_t)0;
      Bf[d][j] = M::from_bits(f);
      Bb[d][j] = M::from_bits(b);
    }
  }
  for (int t = lane; t < 3 * PB; t += 64) sl[wave][t / PB][t % PB] = lam[e * 3 * PB + t];
  const float sxyz = sscale[e * 3 + 0] * sscale[e * 3 + 1] * sscale[e * 3 + 2];

  // gather the extended box (consistent E-vector; outside the domain 0)
  int64_t ex, ey, ez;
  elem_coords(e, nex, ney, ex, ey, ez);
  float mr = 0.f;
  for (int t = lane; t < PB * PB * PB; t += 64) {
    int a = t % PB, b = (t / PB) % PB, c = t / (PB * PB);
    int dx = a == 0 ? -1 : (a == PB - 1 ? 1 : 0), li = a == 0 ? P - 1 : (a == PB - 1 ? 1 : a - 1);
    int dy = b == 0 ? -1 : (b == PB - 1 ? 1 : 0), lj = b == 0 ? P - 1 : (b == PB - 1 ? 1 : b - 1);
    int dz = c == 0 ? -1 : (c == PB - 1 ? 1 : 0), lk = c == 0 ? P - 1 : (c == PB - 1 ? 1 : c - 1);
    bool ok = ex + dx >= 0 && ex + dx < nex && ey + dy >= 0 && ey + dy < ney && ez + dz >= 0 &&
              ez + dz < nez;
    // unconditional load (an outside neighbour reads the element itself, then 0)
    int64_t en = ok ? e + dx + (int64_t)dy * nex + (int64_t)dz * nex * ney : e;
    float v = r[en * N3 + (lk * N + lj) * N + li];
    v = ok ? v : 0.f;
    X[c * PS + b * RS + a] = v;
    mr = fmaxf(mr, fabsf(v));
  }
  mr = wave_max(mr);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  const float inv_r = mr > 0.f ? 1.f / mr : 0.f;

  // one contraction: src (FP32 box) -> dst, along `dir`, with fragment B;
  // `post` receives each accumulator value with its (m, n) before it is stored
  auto contract = [&](const float *src, float *dst, int dir, frag B, float scale, auto &&post) {
    for (int tile = 0; tile < TILES; ++tile) {
      frag A;
      const int m = tile * 16 + col;
      for (int j = 0; j < 4; ++j) {
        int k = kb + j;
        float v = (m < MROWS && k < PB) ? src[box_index<PB, RS, PS>(dir, m, k)] * scale : 0.f;
        A[j] = M::enc(v);
      }
      float4_t acc = {0.f, 0.f, 0.f, 0.f};
      acc = M::mma(A, B, acc);
      // src and dst are distinct buffers, so the stores cannot clobber operands
      for (int j = 0; j < 4; ++j) {
        int mm = tile * 16 + kb + j;
        if (mm < MROWS && col < PB) dst[box_index<PB, RS, PS>(dir, mm, col)] = post(acc[j], mm, col);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  };
  auto id = [](float v, int, int) { return v; };

  contract(X, Y, 0, Bf[0], inv_r, id);   // along x
  contract(Y, X, 1, Bf[1], 1.f, id);     // along y
  // along z, then the diagonal of eq. 9 (rows m = (b, a), column n = c)
  float mt = 0.f;
  auto diag = [&](float v, int m, int n) {
    int b = m / PB, a = m - b * PB;
    float dl = sl[wave][0][a] + sl[wave][1][b] + sl[wave][2][n];
    float s = dl > 0.f ? sxyz * v / dl : 0.f;  // +inf -> 0 (decoupled node)
    mt = fmaxf(mt, fabsf(s));
    return s;
  };
  contract(X, Y, 2, Bf[2], 1.f, diag);
  mt = wave_max(mt);
  const float inv_t = mt > 0.f ? 1.f / mt : 0.f;
  contract(Y, X, 2, Bb[2], inv_t, id);   // back along z
  contract(X, Y, 1, Bb[1], 1.f, id);     // back along y
  // back along x, fused with the RAS restriction to the element's own nodes
  const float fin = sxyz * mr * mt;
  for (int tile = 0; tile < TILES; ++tile) {
    frag A;
    const int m = tile * 16 + col;
    for (int j = 0; j < 4; ++j) {
      int k = kb + j;
      float v = (m < MROWS && k < PB) ? Y[box_index<PB, RS, PS>(0, m, k)] : 0.f;
      A[j] = M::enc(v);
    }
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
    acc = M::mma(A, Bb[0], acc);
    for (int j = 0; j < 4; ++j) {
      int mm = tile * 16 + kb + j;  // (c, b)
      int c = mm / PB, b = mm - c * PB, a = col;
      if constexpr (ASM) {  // whole box to z[E][pb^3]; the overlap sum follows
        if (mm < MROWS && a < PB) z[e * PB * PB * PB + mm * PB + a] = acc[j] * fin;
        continue;
      }
      if (mm < MROWS && a >= 1 && a <= P + 1 && b >= 1 && b <= P + 1 && c >= 1 && c <= P + 1) {
        int64_t o = e * N3 + ((c - 1) * N + (b - 1)) * N + (a - 1);
        z[o] = W[o] * (acc[j] * fin);
      }
    }
  }
}

// Second form: the 16-bit box stays in LDS between contractions, every
// operand fragment is one 8-byte LDS read, and S is the A operand so that a
// contraction's D fragment (lane: 4 consecutive rows, one column) is the B
// fragment of a contraction over those rows.  Tiles are slices of the box
// (16x16, zero padded), one wavefront per element.  Order:
//   x: Y1_c = Sx^T X_c      (slices c,  rows a', cols b)  -> LDS [c][a'][b]
//   y: Y2_c = Sy^T Y1_c^T   (slices c,  rows b', cols a') -> LDS [a'][b'][c]
//   z: Y3_a = Sz^T (...)    (slices a', rows c', cols b'), divide by lambda sums
//   back z from registers: Y4_a = Sz Y3_a (rows c, cols b') -> LDS [a'][c][b']
//   back y: Y5_a = Sy (...) (rows b, cols c)              -> LDS [b][c][a']
//   back x: Y6_b = Sx (...) (rows a, cols c) -> own nodes times the RAS weight
// Each step keeps its PB tiles of accumulators in registers until all reads
// of the previous layout are done, so one LDS buffer per wave suffices.
template <int P, bool BF, bool ASM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_fdm_mfma2(int64_t E, int nex, int ney, int nez,
                                                   const float *__restrict__ r,
                                                   const uint16_t *__restrict__ S16,
                                                   const float *__restrict__ sscale,
                                                   const float *__restrict__ lam,
                                                   const float *__restrict__ W,
                                                   float *__restrict__ z, int nv) {
  using M = Mma<BF>;
  using frag = typename M::frag;
  constexpr int PB = P + 3, N = P + 1, N3 = N * N * N;
  constexpr int RS = 20, SS = 324;  // LDS strides in 16-bit units (8-byte aligned rows)
  // PB slices, and room for the FP32 output staging
  constexpr int OUT = 2 * (ASM ? PB * PB * PB : N3);
  constexpr int BUF = ((PB * SS > OUT ? PB * SS : OUT) + 3) / 4 * 4;
  constexpr int WAVES = 4;
  static_assert(PB <= 16, "pbar must fit one 16-wide tile");
  __shared__ uint16_t lds[WAVES * BUF];
  
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int vec;
  const int64_t e = (int64_t)split_rhs(xcd_block(), nv, vec) * WAVES + wave;
  if (e >= E) return;  // whole wave leaves; no block-wide barriers below
  r += (int64_t)vec * E * N3;  // right side vec (RAS: output E-vectors nloc apart)
  z += (int64_t)vec * E * N3;
  uint16_t *buf = lds + wave * BUF;
  const int g = lane >> 4, t = lane & 15;

  auto bits = [](float x) -> uint16_t {
    auto h = M::enc(x);
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
  };
  // (at is a multiple of 4: one 8-byte LDS read)
  auto load_frag = [&](int at) -> frag { return *reinterpret_cast<const frag *>(buf + at); };
  auto sync = []() {
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  };

  // A fragments of S: forward A[mode][node] = S[node][mode], backward A[node][mode]
  const uint16_t *Se = S16 + e * 3 * PB * PB;
  frag Af[3], Ab[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 4 * g + j;
      const bool ok = k < PB && t < PB;
      Af[d][j] = M::from_bits(ok ? Se[(d * PB + k) * PB + t] : (uint16_t)0);
      Ab[d][j] = M::from_bits(ok ? Se[(d * PB + t) * PB + k] : (uint16_t)0);
    }
  // eigenvalues for eq. 9: lambda_y at this lane's column t, lambda_z at its
  // rows 4g+j (padding: +inf, so that the mode is dropped); lambda_x per tile
  const float *le = lam + e * 3 * PB;
  const float inf = __builtin_huge_valf();
  const float ly = t < PB ? le[PB + t] : inf;
  float lz[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) lz[j] = 4 * g + j < PB ? le[2 * PB + 4 * g + j] : inf;
  const float sxyz = sscale[e * 3 + 0] * sscale[e * 3 + 1] * sscale[e * 3 + 2];

  // zero the buffer (padding rows and columns are read as operands)
  for (int q = lane * 4; q < BUF; q += 256) *reinterpret_cast<uint2 *>(buf + q) = make_uint2(0u, 0u);
  // gather the extended box row by row (row (b, c): the x-neighbours' nodes
  // p-1 and 1 around the element's own N nodes; outside the domain 0), scaled
  // by its largest entry
  int64_t ex, ey, ez;
  elem_coords(e, nex, ney, ex, ey, ez);
  constexpr int NR = (PB * PB + 63) / 64;
  float v[NR][PB];
  float mr = 0.f;
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int row = lane + 64 * u;
    const int rr = row < PB * PB ? row : 0;
    const int b = rr % PB, c = rr / PB;
    const int dy = b == 0 ? -1 : (b == PB - 1 ? 1 : 0), lj = b == 0 ? P - 1 : (b == PB - 1 ? 1 : b - 1);
    const int dz = c == 0 ? -1 : (c == PB - 1 ? 1 : 0), lk = c == 0 ? P - 1 : (c == PB - 1 ? 1 : c - 1);
    const bool okyz = row < PB * PB && ey + dy >= 0 && ey + dy < ney && ez + dz >= 0 && ez + dz < nez;
    const int64_t em = okyz ? e + (int64_t)dy * nex + (int64_t)dz * nex * ney : e;
    const float *src = r + em * N3 + (lk * N + lj) * N;
    const bool okl = okyz && ex > 0, okr = okyz && ex < nex - 1;
    const float left = src[okl ? -N3 + P - 1 : 0], right = src[okr ? N3 + 1 : 0];
    v[u][0] = okl ? left : 0.f;
    v[u][PB - 1] = okr ? right : 0.f;
#pragma unroll
    for (int a = 0; a < N; ++a) v[u][a + 1] = okyz ? src[a] : 0.f;
#pragma unroll
    for (int a = 0; a < PB; ++a) mr = fmaxf(mr, fabsf(v[u][a]));
  }
  mr = wave_max(mr);
  const float inv_r = mr > 0.f ? 1.f / mr : 0.f;
  sync();
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int row = lane + 64 * u;
    if (row < PB * PB) {
      const int b = row % PB, c = row / PB;
#pragma unroll
      for (int a = 0; a < PB; ++a) buf[c * SS + b * RS + a] = bits(v[u][a] * inv_r);
    }
  }
  sync();

  float4_t acc[PB];
  const float4_t zero4 = {0.f, 0.f, 0.f, 0.f};
  // x: tile c, B[a][b] = X[c][b][a]
#pragma unroll
  for (int c = 0; c < PB; ++c) acc[c] = M::mma(Af[0], load_frag(c * SS + t * RS + 4 * g), zero4);
  sync();
#pragma unroll
  for (int c = 0; c < PB; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) buf[c * SS + (4 * g + j) * RS + t] = bits(acc[c][j]);
  sync();
  // y: tile c, B[b][a'] from [c][a'][b]
#pragma unroll
  for (int c = 0; c < PB; ++c) acc[c] = M::mma(Af[1], load_frag(c * SS + t * RS + 4 * g), zero4);
  sync();
  if (t < PB) {  // slice a' = t
#pragma unroll
    for (int c = 0; c < PB; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) buf[t * SS + (4 * g + j) * RS + c] = bits(acc[c][j]);
  }
  sync();
  // z: tile a', B[c][b'] from [a'][b'][c]; then the diagonal of eq. 9
  float mt = 0.f;
#pragma unroll
  for (int a = 0; a < PB; ++a) {
    acc[a] = M::mma(Af[2], load_frag(a * SS + t * RS + 4 * g), zero4);
    const float lxy = le[a] + ly;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float dl = lxy + lz[j];
      const float val = dl > 0.f ? sxyz * acc[a][j] * __builtin_amdgcn_rcpf(dl) : 0.f;  // +inf -> 0
      acc[a][j] = val;
      mt = fmaxf(mt, fabsf(val));
    }
  }
  mt = wave_max(mt);
  const float inv_t = mt > 0.f ? 1.f / mt : 0.f;
  sync();
  // back along z from registers: B[c'][b'] = scaled tile; result [a'][c][b']
#pragma unroll
  for (int a = 0; a < PB; ++a) {
    frag B;
#pragma unroll
    for (int j = 0; j < 4; ++j) B[j] = M::enc(acc[a][j] * inv_t);
    acc[a] = M::mma(Ab[2], B, zero4);
#pragma unroll
    for (int j = 0; j < 4; ++j) buf[a * SS + (4 * g + j) * RS + t] = bits(acc[a][j]);
  }
  sync();
  // back along y: tile a', B[b'][c] from [a'][c][b']; result [b][c][a']
#pragma unroll
  for (int a = 0; a < PB; ++a) acc[a] = M::mma(Ab[1], load_frag(a * SS + t * RS + 4 * g), zero4);
  sync();
#pragma unroll
  for (int a = 0; a < PB; ++a)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * g + j < PB) buf[(4 * g + j) * SS + t * RS + a] = bits(acc[a][j]);  // slice b = 4g+j
  sync();
  // back along x: tile b, B[a'][c] from [b][c][a']; rows a, columns c
#pragma unroll
  for (int b = 0; b < PB; ++b) acc[b] = M::mma(Ab[0], load_frag(b * SS + t * RS + 4 * g), zero4);
  sync();
  // stage the result in LDS (FP32, node order) and write it out in contiguous runs
  const float fin = sxyz * mr * mt;
  float *st = reinterpret_cast<float *>(buf);
  const int c = t;
#pragma unroll
  for (int b = 0; b < PB; ++b)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = 4 * g + j;
      if constexpr (ASM) {
        if (a < PB && c < PB) st[(c * PB + b) * PB + a] = acc[b][j] * fin;
      } else {
        if (a >= 1 && a <= P + 1 && b >= 1 && b <= P + 1 && c >= 1 && c <= P + 1)
          st[((c - 1) * N + (b - 1)) * N + (a - 1)] = acc[b][j] * fin;
      }
    }
  sync();
  if constexpr (ASM) {
    float *zb = z + e * PB * PB * PB;
    for (int q = lane; q < PB * PB * PB; q += 64) zb[q] = st[q];
  } else {
    const int64_t o = e * N3;
    for (int q = lane; q < N3; q += 64) z[o + q] = W[o + q] * st[q];
  }
}

template <int P>
static void fdm_mfma_p(const Ctx &c, const Level &L, const float *r, float *z, bool bf,
                       bool asm_mode, hipStream_t s, int nv) {
  const float *sscale = L.sscale;
  if (asm_mode && nv > 1) {  // one box buffer: right sides in turn
    for (int k = 0; k < nv; ++k) fdm_mfma_p<P>(c, L, r + k * L.nloc, z + k * L.nloc, bf, true, s, 1);
    return;
  }
  unsigned grid = (unsigned)((L.E + 3) / 4 * nv);
  float *out = z;
  if (asm_mode) {
    if (!L.box32) fail(SEM_EINVAL, "ASM box buffer was not built");
    out = L.box32;
  }
#define SEM_MFMA_LAUNCH(BFV, ASMV)                                                                \
  do {                                                                                            \
    if (c.fdm_mfma1)                                                                              \
      hipLaunchKernelGGL((k_fdm_mfma<P, BFV, ASMV>), dim3(grid), dim3(256), 0, s, L.E, c.nex,      \
                         c.ney, c.nez, r, L.S16, sscale, L.lam32, L.w32, out, nv);                 \
    else                                                                                          \
      hipLaunchKernelGGL((k_fdm_mfma2<P, BFV, ASMV>), dim3(grid), dim3(256), 0, s, L.E, c.nex,     \
                         c.ney, c.nez, r, L.S16, sscale, L.lam32, L.w32, out, nv);                 \
  } while (0)
  if (bf && asm_mode) SEM_MFMA_LAUNCH(true, true);
  else if (bf) SEM_MFMA_LAUNCH(true, false);
  else if (asm_mode) SEM_MFMA_LAUNCH(false, true);
  else SEM_MFMA_LAUNCH(false, false);
#undef SEM_MFMA_LAUNCH
  SEM_LAUNCH("k_fdm_mfma");
  if (asm_mode) launch_asm_sum<float>(c, L, L.box32, z, s);
}

// prec < 0: pack the 16-bit factors at setup; otherwise apply (RAS only)
void launch_fdm_mfma(const Ctx &c, const Level &L, const float *r, float *z, bool asm_mode,
                     int prec, hipStream_t s, int nv) {
  if (!L.S16 || !L.S32) fail(SEM_EINVAL, "16-bit FDM data were not built");
  const bool bf = (prec < 0 ? c.fdm_prec : prec) == SEM_BF16;
  if (prec < 0) {
    float *sscale = L.sscale;
    int64_t tasks = 3 * L.E;
    hipLaunchKernelGGL(k_fdm_pack16, dim3((unsigned)((tasks + 63) / 64)), dim3(64), 0, s, L.E,
                       L.pb, L.S32, L.S16, sscale, bf ? 1 : 0);
    SEM_LAUNCH("k_fdm_pack16");
    return;
  }
  switch (L.p) {
    case 2: fdm_mfma_p<2>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 3: fdm_mfma_p<3>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 4: fdm_mfma_p<4>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 5: fdm_mfma_p<5>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 6: fdm_mfma_p<6>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 7: fdm_mfma_p<7>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 8: fdm_mfma_p<8>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 9: fdm_mfma_p<9>(c, L, r, z, bf, asm_mode, s, nv); break;
    case 10: fdm_mfma_p<10>(c, L, r, z, bf, asm_mode, s, nv); break;
    default: fail(SEM_EUNSUPPORTED, "MFMA FDM: unsupported degree");
  }
}

}  // namespace sem
