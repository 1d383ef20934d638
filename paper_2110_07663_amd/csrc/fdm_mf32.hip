// RAS local solves by the fast diagonalisation method (Sec. 2.2.2, eqs. 8-9)
// on the matrix cores: FP32 operands, or FP16 / BF16 operands with FP32
// accumulation (k_fdm_mf16, the same kernel forms with v_mfma_f32_4x4x4).
//
// Each of the six 1D contractions of the (p+3)^3 box is a product of the box
// lines with a (p+3)x(p+3) factor: out[line][m] = sum_k in[line][k] S[k][m].
// A lane owns one line (in each pass of one wavefront, lines 64s + lane of
// slot s) and v_mfma_f32_4x4x1 forms four outputs of all 64 lines at a time:
// its 16 blocks (4 lanes each) all take the same four-entry A operand, read
// from one block by the broadcast controls (CBSZ = 4, ABID = q), and their own
// lanes' line values as B, so register i of lane l receives
// out[line of l][4g + i].  One register then carries the A operands of 16
// (k, g) pairs, lane 4q + i holding S[k][4g + i], and a whole factor fits in
// two or three registers loaded once per element.  Against the FP32 vector
// pipe (one multiply-add per lane and cycle without packed instructions) the
// matrix core does four per lane in the same time, at the cost of padding the
// modes to a multiple of 4.
//
// One wavefront per element, four per workgroup; the waves of a workgroup
// meet at a barrier only in the form that sums their shared x-faces before
// the store (XF).  The first pass reads its x-lines straight from the
// E-vector through range-checked buffer loads (the element's own row and one
// node of each x-neighbour; zeros outside the domain); every later pass reads
// lines that the previous pass wrote contiguously into the wave's LDS buffer
// (16-byte reads).  The z pass divides by the eigenvalue sums of eq. 9 in
// registers and goes straight back along z; the backward passes form only the
// nodes RAS keeps, and the last one writes the element's rows times the RAS
// weight.  The 16-bit forms take four k per instruction (84 instead of 280
// matrix instructions per element at p = 7); their operands are kept in range
// by powers of two (the box, and the eigenvalue-scaled tensor, over their
// largest entry) and by factors stored over their largest entries.
#include "sem_internal.h"

namespace sem {

namespace {

typedef float mf4_t __attribute__((ext_vector_type(4)));

// D += A_q (x) B on the 16 blocks, A broadcast from block q (a constant once
// the loops are unrolled)
__device__ __attribute__((always_inline)) inline mf4_t mfma_bq(float a, float b, mf4_t c, int q) {
  switch (q) {
    case 0: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 0, 0);
    case 1: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 1, 0);
    case 2: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 2, 0);
    case 3: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 3, 0);
    case 4: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 4, 0);
    case 5: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 5, 0);
    case 6: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 6, 0);
    case 7: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 7, 0);
    case 8: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 8, 0);
    case 9: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 9, 0);
    case 10: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 10, 0);
    case 11: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 11, 0);
    case 12: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 12, 0);
    case 13: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 13, 0);
    case 14: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 14, 0);
    default: return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, 15, 0);
  }
}

// Operand formats of the contractions: FP32 (v_mfma_f32_4x4x1, one k per
// instruction) or FP16 / BF16 (v_mfma_f32_4x4x4, four k per instruction, FP32
// accumulation).  In the 16-bit forms lane 4q + i of the broadcast block holds
// four consecutive k of row i of A, and lane 4b + j four consecutive k of
// column j of B (its line), packed two per register.
enum : int { kOpF32 = 0, kOpF16 = 1, kOpBF16 = 2 };
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));  // four 16-bit operands
typedef float f2_t __attribute__((ext_vector_type(2)));

template <int OP>
__device__ inline uint32_t pack2(float a, float b) {  // round to nearest even
  if constexpr (OP == kOpF16) {
    typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{a, b}, h2_t));
  } else {
    typedef __bf16 b2_t __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{a, b}, b2_t));
  }
}

template <int OP, int Q>
__device__ __attribute__((always_inline)) inline mf4_t mfma16_q(u2_t a, u2_t b, mf4_t c) {
  typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
  typedef short s4_t __attribute__((ext_vector_type(4)));
  if constexpr (OP == kOpF16)
    return __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(h4_t, a),
                                              __builtin_bit_cast(h4_t, b), c, 4, Q, 0);
  else
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(s4_t, a),
                                                  __builtin_bit_cast(s4_t, b), c, 4, Q, 0);
}
// D += A_q B (four k) on the 16 blocks, A broadcast from block q
template <int OP>
__device__ __attribute__((always_inline)) inline mf4_t mfma16(u2_t a, u2_t b, mf4_t c, int q) {
  switch (q) {
    case 0: return mfma16_q<OP, 0>(a, b, c);
    case 1: return mfma16_q<OP, 1>(a, b, c);
    case 2: return mfma16_q<OP, 2>(a, b, c);
    case 3: return mfma16_q<OP, 3>(a, b, c);
    case 4: return mfma16_q<OP, 4>(a, b, c);
    case 5: return mfma16_q<OP, 5>(a, b, c);
    case 6: return mfma16_q<OP, 6>(a, b, c);
    case 7: return mfma16_q<OP, 7>(a, b, c);
    case 8: return mfma16_q<OP, 8>(a, b, c);
    case 9: return mfma16_q<OP, 9>(a, b, c);
    case 10: return mfma16_q<OP, 10>(a, b, c);
    case 11: return mfma16_q<OP, 11>(a, b, c);
    case 12: return mfma16_q<OP, 12>(a, b, c);
    case 13: return mfma16_q<OP, 13>(a, b, c);
    case 14: return mfma16_q<OP, 14>(a, b, c);
    default: return mfma16_q<OP, 15>(a, b, c);
  }
}

// the largest of the lanes' values over the wavefront (the callers pass
// each lane's largest |entry|)
__device__ inline float wave_absmax(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
// 2^-e with m = f 2^e, 0.5 <= f < 1: a scale that brings m into [0.5, 1)
// exactly (0 for m = 0)
__device__ inline float pow2_below(float m, int &e) {
  e = __builtin_amdgcn_frexp_expf(m);
  return m > 0.f ? __builtin_amdgcn_ldexpf(1.0f, -e) : 0.f;
}

// The RAS weight of an element's own node (Sec. 2.2.2: mask / multiplicity,
// node_w1 per direction) is exact in FP32 and equal to the assembled weight,
// so from p = 4 on the solve computes it instead of loading it (at p <= 3
// the element's rows are short and one load costs less than the arithmetic:
// 21.0 against 23.8 us per launch at p = 3).  bcm: bit f set when domain
// face f (x-, x+, y-, y+, z-, z+) is Dirichlet; w: the stored weights
// (an E-vector), read at p <= 3.
struct RasW {
  int nex, ney, nez, bcm;
  const float *w;
};
template <int P>
constexpr bool kRasWComputed = P >= 4;

template <int P>
struct Mf {
  static constexpr int PB = P + 3, N = P + 1, N3 = N * N * N;
  static constexpr int NL = PB * PB, SF = (NL + 63) / 64;  // forward lines, slots
  static constexpr int MG = (PB + 3) / 4;                  // groups of 4 modes
  static constexpr int KG = (N + 3) / 4;                   // groups of 4 kept nodes
  static constexpr int LS = (PB + 3) / 4 * 4;              // LDS line stride
  static constexpr int QF = PB * MG, QB = PB * KG;         // A operands per pass
  static constexpr int UF = (QF + 15) / 16, UB = (QB + 15) / 16;
  static constexpr int NLY = PB * N, SY = (NLY + 63) / 64;  // backward y lines (kept planes)
  static constexpr int NLX = N * N, SX = (NLX + 63) / 64;   // backward x lines (kept rows)
  static constexpr int BUF = NL * LS;                        // floats per wavefront
  static constexpr int WAVES = 4;
  // 16-bit operands: k in groups of four (forward: the line's nodes; backward:
  // the modes), one register pair of A operands per direction and pass kind
  static constexpr int K4 = (PB + 3) / 4;
  static constexpr int QF16 = K4 * MG, QB16 = K4 * KG;
  static_assert(QF16 <= 16 && QB16 <= 16, "16-bit A operands exceed one broadcast register");
  static_assert(K4 == MG, "16-bit forward pairs: k groups and mode groups both cover PB");
};

// 1 / (lambda_x + lambda_y + lambda_z): +inf (a decoupled node) gives 0.  A
// zero sum (the constant mode of a box floating on Neumann faces in all three
// directions) cannot occur here: the launcher sends such meshes to the vector
// kernel, which drops that mode.
__device__ inline float mf_inv(float d) { return __builtin_amdgcn_rcpf(d); }

// Raw-buffer view of an FP32 array: a load at a byte offset at or past nbytes
// returns zero (the range check of the buffer instructions).  The box gather
// reads the nodes outside the domain, and the A operands their zero padding,
// through such offsets instead of selecting zeros after the loads.
constexpr uint32_t kOutside = 0x80000000u;  // past every buffer window used here
constexpr uint32_t kWindowMax = 0x7FFFFF00u;
struct BufF32 {
  __amdgpu_buffer_rsrc_t rsrc;
  __device__ BufF32(const float *p, uint32_t nbytes)
      : rsrc(__builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, (int)nbytes,
                                               0x00020000)) {}
  __device__ float ld(uint32_t off) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rsrc, off, 0, 0));
  }
  __device__ f2_t ld2(uint32_t off) const {  // off a multiple of 8
    return __builtin_bit_cast(f2_t, __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0));
  }
  __device__ mf4_t ld4(uint32_t off) const {
    return __builtin_bit_cast(mf4_t, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
  }
};

// forward contraction of one slot: acc[g][i] = sum_k v[k] S[k][4g + i]
template <int P>
__device__ __attribute__((always_inline)) inline void mf_forward(const float *A, const float *v,
                                                                 mf4_t *acc) {
  using F = Mf<P>;
#pragma unroll
  for (int g = 0; g < F::MG; ++g) acc[g] = mf4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < F::PB; ++k)
#pragma unroll
    for (int g = 0; g < F::MG; ++g) {
      const int q = k * F::MG + g;
      acc[g] = mfma_bq(A[q >> 4], v[k], acc[g], q & 15);
    }
}

// backward contraction to the kept nodes: acc[g][i] = sum_m S[1 + 4g + i][m] h[m]
template <int P>
__device__ __attribute__((always_inline)) inline void mf_backward(const float *A, const float *h,
                                                                  mf4_t *acc) {
  using F = Mf<P>;
#pragma unroll
  for (int g = 0; g < F::KG; ++g) acc[g] = mf4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < F::PB; ++m)
#pragma unroll
    for (int g = 0; g < F::KG; ++g) {
      const int q = m * F::KG + g;
      acc[g] = mfma_bq(A[q >> 4], h[m], acc[g], q & 15);
    }
}

// the 16-bit forms of the two contractions: the B operands are the line's
// values (times sc when SC), four k per operand, zero past PB
template <int P, int OP, bool SC>
__device__ __attribute__((always_inline)) inline void mf16_operands(const float *v, float sc,
                                                                     u2_t *b) {
  using F = Mf<P>;
  auto at = [&](int k) { return k < F::PB ? (SC ? v[k] * sc : v[k]) : 0.f; };
#pragma unroll
  for (int kg = 0; kg < F::K4; ++kg)
    b[kg] = u2_t{pack2<OP>(at(4 * kg), at(4 * kg + 1)), pack2<OP>(at(4 * kg + 2), at(4 * kg + 3))};
}
template <int P, int OP, bool SC>
__device__ __attribute__((always_inline)) inline void mf16_forward(u2_t A, const float *v,
                                                                   float sc, mf4_t *acc) {
  using F = Mf<P>;
  u2_t b[F::K4];
  mf16_operands<P, OP, SC>(v, sc, b);
#pragma unroll
  for (int g = 0; g < F::MG; ++g) acc[g] = mf4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kg = 0; kg < F::K4; ++kg)
#pragma unroll
    for (int g = 0; g < F::MG; ++g) acc[g] = mfma16<OP>(A, b[kg], acc[g], kg * F::MG + g);
}
template <int P, int OP, bool SC>
__device__ __attribute__((always_inline)) inline void mf16_backward(u2_t A, const float *h,
                                                                    float sc, mf4_t *acc) {
  using F = Mf<P>;
  u2_t b[F::K4];
  mf16_operands<P, OP, SC>(h, sc, b);
#pragma unroll
  for (int g = 0; g < F::KG; ++g) acc[g] = mf4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mg = 0; mg < F::K4; ++mg)
#pragma unroll
    for (int g = 0; g < F::KG; ++g) acc[g] = mfma16<OP>(A, b[mg], acc[g], mg * F::KG + g);
}

template <int P>
__device__ __attribute__((always_inline)) inline void mf_read_line(const float *buf, int line,
                                                                   float *v) {
  using F = Mf<P>;
  const mf4_t *src = reinterpret_cast<const mf4_t *>(buf + line * F::LS);
#pragma unroll
  for (int q = 0; q < F::LS / 4; ++q) {
    const mf4_t t = src[q];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * q + i < F::PB) v[4 * q + i] = t[i];
  }
}

// orders the LDS traffic of one wavefront between passes (global loads in
// flight, such as the next element's box, are not waited for)
__device__ inline void mf_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) only
  __builtin_amdgcn_wave_barrier();
}

// What one element's solve reads from global memory, loaded ahead of its use:
// the x-lines of the box (the element's own row of a y/z neighbour or itself,
// and one node of each x-neighbour; RS: also those of the subtrahend), zero
// where they lie outside the domain, the A operands of its first four passes
// and the eigenvalue sums of the z pass (what the last two passes read comes
// later, mf_load_late).
// XS = 1 (r) or 2 (rs): that input comes from A with the x step of its
// gather-scatter left out (its y and z steps done), so the x-neighbours'
// copies of the row's end nodes (their nodes p and 0) are read as well and
// added: each copy of a node then holds the sum over all its copies, as
// after the whole gather-scatter (the x step taken last).
// YS: that input also comes without the y step (only the z step done): the
// rows on the element's y-faces (own rows j = 0, p of the element and of its
// z-neighbours) also read the y-neighbour's copy of the row, of its end nodes'
// x-partners and of the halo nodes beside it, and add them (y, then x).
template <int P, bool RS, int XS, bool YS>
struct MfIn {
  using F = Mf<P>;
  float own[F::SF][F::N], lft[F::SF], rgt[F::SF];
  float sown[RS ? F::SF : 1][RS ? F::N : 1], slft[RS ? F::SF : 1], srgt[RS ? F::SF : 1];
  float xlp[XS ? F::SF : 1], xrp[XS ? F::SF : 1];  // x-partner copies of nodes 0 and p
  static constexpr int YSF = YS ? F::SF : 1;
  float yrow[YSF][YS ? F::N : 1];  // y-partner copy of the row
  float yxl[YSF], yxr[YSF];        // ... of the x-partners of its nodes 0 and p
  float ylf[YSF], yrg[YSF];        // ... of the halo nodes (left node p-1, right node 1)
  float Af[3][F::UF], Ab[3][F::UB];
  u2_t Af16[3], Ab16z;       // 16-bit forms: forward and z backward A operands (factors / s_d)
  float lxy[F::SF];          // lambda_x + lambda_y of the slot's z-line
};

// Raw-buffer view of the packed 16-bit A operands (zero at or past nbytes)
struct BufU2 {
  __amdgpu_buffer_rsrc_t rsrc;
  __device__ BufU2(const uint32_t *p, uint32_t nbytes)
      : rsrc(__builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(p), (short)0, (int)nbytes,
                                               0x00020000)) {}
  __device__ u2_t ld(uint32_t off) const {
    return __builtin_bit_cast(u2_t, __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0));
  }
};

template <int P, bool RS, int XS, bool YS, int OP = kOpF32>
__device__ __attribute__((always_inline)) inline void mf_load(
    MfIn<P, RS, XS, YS> &in, int64_t e, int nex, int ney, int nez, const BufF32 &r, const BufF32 &rs,
    int64_t eb, const float *__restrict__ Sg, const float *__restrict__ lamg,
    const RasW &W, int lane, const uint32_t *__restrict__ A16 = nullptr,
    const float *__restrict__ ssc = nullptr) {
  using F = Mf<P>;
  constexpr int PB = F::PB, N = F::N, N3 = F::N3, MG = F::MG, KG = F::KG;
  if constexpr (OP != kOpF32) {
    // 16-bit A operands, packed at setup in lane order (k_fdm_mf16_pack): the
    // lanes of the forward pairs, then those of the backward pairs, per
    // direction; the other lanes read zeros
    constexpr int NF = 4 * F::QF16, NE = 4 * (F::QF16 + F::QB16);
    const BufU2 At(A16 + e * 3 * NE * 2, 3 * NE * 8);
#pragma unroll
    for (int d = 0; d < 3; ++d)
      in.Af16[d] = At.ld(lane < NF ? (uint32_t)(d * NE + lane) * 8 : kOutside);
    in.Ab16z = At.ld(lane < NE - NF ? (uint32_t)(2 * NE + NF + lane) * 8 : kOutside);
    // (what the last two passes read is loaded by the solve once its first
    // pass is issued)
  } else {
  const BufF32 Se(Sg + e * 3 * PB * PB, 3 * PB * PB * 4);  // the element's three factors
  // A operands: forward (k, g) -> lane 4q + i holds S_d[k][4g + i]; backward
  // (m, g) -> S_d[1 + 4g + i][m]; zero where the index runs past the factor
  {
    const int i = lane & 3, qb = lane >> 2;
#pragma unroll
    for (int u = 0; u < F::UF; ++u) {
      const int q = 16 * u + qb, k = q / MG, m = 4 * (q % MG) + i;
      const uint32_t at = q < F::QF && m < PB ? (uint32_t)(k * PB + m) * 4 : kOutside;
#pragma unroll
      for (int d = 0; d < 3; ++d) in.Af[d][u] = Se.ld(at + d * PB * PB * 4);
    }
#pragma unroll
    for (int u = 0; u < F::UB; ++u) {
      const int q = 16 * u + qb, m = q / KG, k = 1 + 4 * (q % KG) + i;
      const uint32_t at = q < F::QB && k <= N ? (uint32_t)(k * PB + m) * 4 : kOutside;
      in.Ab[2][u] = Se.ld(at + 2 * PB * PB * 4);  // (x and y: loaded by the solve)
    }
  }
  }
  // eigenvalue sums of the z pass (line (a', b') of slot s)
  {
    const float *le = lamg + e * 3 * PB;
#pragma unroll
    for (int s = 0; s < F::SF; ++s) {
      const int l = 64 * s + lane, lc = l < F::NL ? l : 0;
      in.lxy[s] = le[lc % PB] + le[PB + lc / PB];
    }
  }
  int64_t ex, ey, ez;
  elem_coords(e, nex, ney, ex, ey, ez);
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    const int l = 64 * s + lane;
    const int b = l % PB, c = l / PB;
    const int dy = b == 0 ? -1 : (b == PB - 1 ? 1 : 0), lj = b == 0 ? P - 1 : (b == PB - 1 ? 1 : b - 1);
    const int dz = c == 0 ? -1 : (c == PB - 1 ? 1 : 0), lk = c == 0 ? P - 1 : (c == PB - 1 ? 1 : c - 1);
    const bool okyz = l < F::NL && ey + dy >= 0 && ey + dy < ney && ez + dz >= 0 && ez + dz < nez;
    const bool okl = okyz && ex > 0, okr = okyz && ex < nex - 1;
    // the row's byte offset from element eb (at most a plane and a line below e)
    const uint32_t em = (uint32_t)(e - eb) + dy * nex + dz * nex * ney;
    const uint32_t row = (em * N3 + (lk * N + lj) * N) * 4;
    const uint32_t orow = okyz ? row : kOutside;
    const uint32_t il = okl ? row - (N3 - P + 1) * 4 : kOutside;  // left neighbour's node p-1
    const uint32_t ir = okr ? row + (N3 + 1) * 4 : kOutside;      // right neighbour's node 1
    // odd p: a neighbour's halo node and its x-partner node are adjacent and
    // 8-byte aligned (even p - 1), one load for both
    constexpr bool PAIR = P % 2 == 1 && XS == 1;
    if constexpr (PAIR) {
      const f2_t lp = r.ld2(il);                            // left neighbour's nodes p-1, p
      const f2_t rp = r.ld2(okr ? row + N3 * 4 : kOutside);  // right neighbour's nodes 0, 1
      in.lft[s] = lp[0];
      in.xlp[s] = lp[1];
      in.xrp[s] = rp[0];
      in.rgt[s] = rp[1];
    } else {
      in.lft[s] = r.ld(il);
      in.rgt[s] = r.ld(ir);
    }
    if constexpr (XS != 0) {
      const BufF32 &xs = XS == 1 ? r : rs;
      if constexpr (!PAIR) {
        in.xlp[s] = xs.ld(okl ? row - (N3 - P) * 4 : kOutside);  // left neighbour's node p
        in.xrp[s] = xs.ld(okr ? row + N3 * 4 : kOutside);        // right neighbour's node 0
      }
      if constexpr (YS) {
        // own row j = 0 (b = 1) pairs with row j = p of the element below in
        // y, row j = p (b = PB - 2) with row j = 0 of the one above
        const bool ylo = okyz && b == 1 && ey > 0, yhi = okyz && b == PB - 2 && ey < ney - 1;
        const uint32_t ystep = ((uint32_t)nex * N3 - P * N) * 4;
        const bool yp = ylo || yhi;
        const uint32_t yr = ylo ? row - ystep : (yhi ? row + ystep : 0u);
        const uint32_t yrow = yp ? yr : kOutside;
        if constexpr (N % 4 == 0) {
#pragma unroll
          for (int q = 0; q < N / 4; ++q) {
            const mf4_t t = xs.ld4(yrow + 16 * q);
#pragma unroll
            for (int i = 0; i < 4; ++i) in.yrow[s][4 * q + i] = t[i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < N; ++i) in.yrow[s][i] = xs.ld(yrow + 4 * i);
        }
        const bool yl = yp && ex > 0, yh = yp && ex < nex - 1;
        if constexpr (PAIR) {
          const f2_t lp = xs.ld2(yl ? yr - (N3 - P + 1) * 4 : kOutside);
          const f2_t rp = xs.ld2(yh ? yr + N3 * 4 : kOutside);
          in.ylf[s] = lp[0];
          in.yxl[s] = lp[1];
          in.yxr[s] = rp[0];
          in.yrg[s] = rp[1];
        } else {
          in.yxl[s] = xs.ld(yl ? yr - (N3 - P) * 4 : kOutside);
          in.yxr[s] = xs.ld(yh ? yr + N3 * 4 : kOutside);
          in.ylf[s] = xs.ld(yl ? yr - (N3 - P + 1) * 4 : kOutside);
          in.yrg[s] = xs.ld(yh ? yr + (N3 + 1) * 4 : kOutside);
        }
      }
    }
    if constexpr (N % 4 == 0) {
#pragma unroll
      for (int q = 0; q < N / 4; ++q) {
        const mf4_t t = r.ld4(orow + 16 * q);
#pragma unroll
        for (int i = 0; i < 4; ++i) in.own[s][4 * q + i] = t[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i) in.own[s][i] = r.ld(orow + 4 * i);
    }
    if constexpr (RS) {
      in.slft[s] = rs.ld(il);
      in.srgt[s] = rs.ld(ir);
      if constexpr (N % 4 == 0) {
#pragma unroll
        for (int q = 0; q < N / 4; ++q) {
          const mf4_t t = rs.ld4(orow + 16 * q);
#pragma unroll
          for (int i = 0; i < 4; ++i) in.sown[s][4 * q + i] = t[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < N; ++i) in.sown[s][i] = rs.ld(orow + 4 * i);
      }
    }
  }
}

// the local solve of element e from its loaded inputs; buf = the wave's LDS.
// XF: the workgroup's four waves hold four consecutive elements along x, and
// the copies on the three x-faces between them are summed (through xfx, LDS
// shared by the workgroup) before the store, each pair as (p-face + 0-face),
// the order of the gather-scatter's x step, which then covers only the faces
// between workgroups.
// What the last two passes read, loaded once the first pass is issued, so
// that fewer registers are live while the box arrives (at p = 7: 78 instead of
// 85 for the x/y-step form, 6 wavefronts per SIMD instead of 5): the y and x
// backward A operands, the 16-bit forms' factor scales s_d, and the RAS
// weights of the output rows
template <int P>
struct MfLate {
  using F = Mf<P>;
  float Ab[2][F::UB];  // FP32 operands
  u2_t Ab16[2];        // 16-bit operands
  float ssc[3];
  mf4_t wrow[F::SX][F::KG];
};
template <int P, int OP>
__device__ __attribute__((always_inline)) inline void mf_load_late(
    MfLate<P> &lt, int64_t e, const float *__restrict__ Sg, const RasW &W,
    const uint32_t *__restrict__ A16, const float *__restrict__ ssc, int lane) {
  using F = Mf<P>;
  constexpr int PB = F::PB, N = F::N, N3 = F::N3, KG = F::KG;
  if constexpr (OP != kOpF32) {
    constexpr int NF = 4 * F::QF16, NE = 4 * (F::QF16 + F::QB16);
    const BufU2 At(A16 + e * 3 * NE * 2, 3 * NE * 8);
#pragma unroll
    for (int d = 0; d < 2; ++d)
      lt.Ab16[d] = At.ld(lane < NE - NF ? (uint32_t)(d * NE + NF + lane) * 8 : kOutside);
#pragma unroll
    for (int d = 0; d < 3; ++d) lt.ssc[d] = ssc[e * 3 + d];
  } else {
    const BufF32 Se(Sg + e * 3 * PB * PB, 3 * PB * PB * 4);
    const int i = lane & 3, qb = lane >> 2;
#pragma unroll
    for (int u = 0; u < F::UB; ++u) {
      const int q = 16 * u + qb, m = q / KG, k = 1 + 4 * (q % KG) + i;
      const uint32_t at = q < F::QB && k <= N ? (uint32_t)(k * PB + m) * 4 : kOutside;
#pragma unroll
      for (int d = 0; d < 2; ++d) lt.Ab[d][u] = Se.ld(at + d * PB * PB * 4);
    }
  }
  if constexpr (kRasWComputed<P>) {
    int64_t ex, ey, ez;
    elem_coords(e, W.nex, W.ney, ex, ey, ez);
#pragma unroll
    for (int s = 0; s < F::SX; ++s) {
      const int l = 64 * s + lane, lc = l < F::NLX ? l : 0;
      const int j = lc % N, k = lc / N;
      const float wjk = node_w1(j, N, ey, W.ney, W.bcm, 2) * node_w1(k, N, ez, W.nez, W.bcm, 4);
#pragma unroll
      for (int g = 0; g < F::KG; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          lt.wrow[s][g][i] = 4 * g + i < N ? wjk * node_w1(4 * g + i, N, ex, W.nex, W.bcm, 0) : 0.f;
    }
  } else {
#pragma unroll
    for (int s = 0; s < F::SX; ++s) {
      const int l = 64 * s + lane, lc = l < F::NLX ? l : 0;
      const int64_t row = e * N3 + (int64_t)lc * N;
#pragma unroll
      for (int g = 0; g < F::KG; ++g) {
        if constexpr (N % 4 == 0) {
          lt.wrow[s][g] = *reinterpret_cast<const mf4_t *>(W.w + row + 4 * g);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            lt.wrow[s][g][i] = 4 * g + i < N ? W.w[row + 4 * g + i] : 0.f;
        }
      }
    }
  }
}

// 16-bit operands (OP): the factors are stored over their largest entries s_d
// and the output is scaled back by (s_x s_y s_z)^2.  FP16 has a narrow
// exponent range, so there the element's box is also brought into [0.5, 1)
// by a power of two from its largest entry before the forward passes, and the
// eigenvalue-scaled tensor likewise before the backward passes (the output
// then takes both powers of two back); BF16 keeps FP32's exponent range and
// needs neither.
template <int P, bool RS, int XS, bool YS, bool XF, int OP = kOpF32>
__device__ __attribute__((always_inline)) inline void mf_solve(
    const MfIn<P, RS, XS, YS> &in, int64_t e, const float *__restrict__ lamg, float *__restrict__ z,
    float *buf, int lane, float *xfx, int wave, const float *__restrict__ Sg,
    const RasW &W, const uint32_t *__restrict__ A16 = nullptr,
    const float *__restrict__ ssc = nullptr) {
  using F = Mf<P>;
  constexpr int PB = F::PB, N = F::N, N3 = F::N3, LS = F::LS, MG = F::MG, KG = F::KG;
  const float *le = lamg + e * 3 * PB;
  float v[F::SF][PB];
  mf4_t acc[F::SF][MG];
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    // entries outside the domain were loaded as zeros; the deferred steps
    // act on r (XS = 1) or on rs (XS = 2): the y step on the row and its halo
    // nodes, then the x step on the end nodes (as (own + y) + (x + xy))
    float ro[N], so[N], rl = in.lft[s], rr = in.rgt[s], sl = 0.f, sr = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      ro[i] = in.own[s][i];
      so[i] = 0.f;
      if constexpr (RS) so[i] = in.sown[s][i];
    }
    if constexpr (RS) {
      sl = in.slft[s];
      sr = in.srgt[s];
    }
    auto steps = [&](float(&o)[N], float &hl, float &hr) {
      float xl = in.xlp[s], xr = in.xrp[s];
      if constexpr (YS) {
#pragma unroll
        for (int i = 0; i < N; ++i) o[i] += in.yrow[s][i];
        hl += in.ylf[s];
        hr += in.yrg[s];
        xl += in.yxl[s];
        xr += in.yxr[s];
      }
      o[0] += xl;
      o[N - 1] += xr;
    };
    if constexpr (XS == 1) steps(ro, rl, rr);
    if constexpr (XS == 2) steps(so, sl, sr);
    v[s][0] = RS ? rl - sl : rl;
    v[s][PB - 1] = RS ? rr - sr : rr;
#pragma unroll
    for (int i = 0; i < N; ++i) v[s][i + 1] = RS ? ro[i] - so[i] : ro[i];
  }

  int e_in = 0, e_h = 0;
  float sc_in = 1.f;
  constexpr bool NORM = OP == kOpF16;  // range scaling of the 16-bit operands
  if constexpr (NORM) {
    float m = 0.f;
#pragma unroll
    for (int s = 0; s < F::SF; ++s)
#pragma unroll
      for (int k = 0; k < PB; ++k) m = fmaxf(m, fabsf(v[s][k]));
    sc_in = pow2_below(wave_absmax(m), e_in);
  }

  // x: line (b, c) -> modes a'; written as y-lines (a', c), position b
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    if constexpr (OP != kOpF32)
      mf16_forward<P, OP, NORM>(in.Af16[0], v[s], sc_in, acc[s]);
    else
      mf_forward<P>(in.Af[0], v[s], acc[s]);
  }
  MfLate<P> lt;
  mf_load_late<P, OP>(lt, e, Sg, W, A16, ssc, lane);
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    const int l = 64 * s + lane;
    if (l < F::NL) {
      const int b = l % PB, c = l / PB;
#pragma unroll
      for (int g = 0; g < MG; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < PB) buf[(4 * g + i + PB * c) * LS + b] = acc[s][g][i];
    }
  }
  mf_sync();

  // y: line (a', c) -> modes b'; written as z-lines (a', b'), position c
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    const int l = 64 * s + lane;
    mf_read_line<P>(buf, l < F::NL ? l : 0, v[s]);
  }
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    if constexpr (OP != kOpF32)
      mf16_forward<P, OP, false>(in.Af16[1], v[s], 1.f, acc[s]);
    else
      mf_forward<P>(in.Af[1], v[s], acc[s]);
  }
  mf_sync();
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    const int l = 64 * s + lane;
    if (l < F::NL) {
      const int a = l % PB, c = l / PB;
#pragma unroll
      for (int g = 0; g < MG; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < PB) buf[(a + PB * (4 * g + i)) * LS + c] = acc[s][g][i];
    }
  }
  mf_sync();

  // z: line (a', b') -> modes c'; divide by lambda_x + lambda_y + lambda_z;
  // back along z to the kept planes k = 1..N, written as y-lines (a', k), position b'
  mf4_t bk[F::SF][KG];
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    const int l = 64 * s + lane;
    mf_read_line<P>(buf, l < F::NL ? l : 0, v[s]);
  }
  if constexpr (OP != kOpF32) {
    float h[F::SF][PB], m = 0.f;
#pragma unroll
    for (int s = 0; s < F::SF; ++s) {
      mf16_forward<P, OP, false>(in.Af16[2], v[s], 1.f, acc[s]);
      const float lxy = in.lxy[s];
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        h[s][k] = acc[s][k >> 2][k & 3] * mf_inv(lxy + le[2 * PB + k]);
        if constexpr (NORM) m = fmaxf(m, fabsf(h[s][k]));
      }
    }
    float sc_h = 1.f;
    if constexpr (NORM) sc_h = pow2_below(wave_absmax(m), e_h);
#pragma unroll
    for (int s = 0; s < F::SF; ++s) mf16_backward<P, OP, NORM>(in.Ab16z, h[s], sc_h, bk[s]);
  } else {
#pragma unroll
    for (int s = 0; s < F::SF; ++s) {
      mf_forward<P>(in.Af[2], v[s], acc[s]);
      const float lxy = in.lxy[s];
      float h[PB];
#pragma unroll
      for (int m = 0; m < PB; ++m) h[m] = acc[s][m >> 2][m & 3] * mf_inv(lxy + le[2 * PB + m]);
      mf_backward<P>(in.Ab[2], h, bk[s]);
    }
  }
  mf_sync();
#pragma unroll
  for (int s = 0; s < F::SF; ++s) {
    const int l = 64 * s + lane;
    if (l < F::NL) {
      const int a = l % PB, b = l / PB;
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < N) buf[(a + PB * (4 * g + i)) * LS + b] = bk[s][g][i];
    }
  }
  mf_sync();

  // back along y: line (a', k) -> kept rows j = 1..N, written as x-lines (j, k), position a'
  float w[F::SY][PB];
  mf4_t by[F::SY][KG];
#pragma unroll
  for (int s = 0; s < F::SY; ++s) {
    const int l = 64 * s + lane;
    mf_read_line<P>(buf, l < F::NLY ? l : 0, w[s]);
  }
#pragma unroll
  for (int s = 0; s < F::SY; ++s) {
    if constexpr (OP != kOpF32)
      mf16_backward<P, OP, false>(lt.Ab16[1], w[s], 1.f, by[s]);
    else
      mf_backward<P>(lt.Ab[1], w[s], by[s]);
  }
  mf_sync();
#pragma unroll
  for (int s = 0; s < F::SY; ++s) {
    const int l = 64 * s + lane;
    if (l < F::NLY) {
      const int a = l % PB, k = l / PB;
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < N) buf[(4 * g + i + N * k) * LS + a] = by[s][g][i];
    }
  }
  mf_sync();

  // back along x: line (j, k) -> kept nodes i = 1..N: the element's row (j, k)
  // times the RAS weight
  mf4_t o[F::SX][KG];
  float osc = 1.f;
  if constexpr (OP != kOpF32) {
    const float s3 = lt.ssc[0] * lt.ssc[1] * lt.ssc[2];
    osc = __builtin_amdgcn_ldexpf(s3 * s3, e_in + e_h);
  }
#pragma unroll
  for (int s = 0; s < F::SX; ++s) {
    const int l = 64 * s + lane;
    float u[PB];
    mf4_t bx[KG];
    mf_read_line<P>(buf, l < F::NLX ? l : 0, u);
    if constexpr (OP != kOpF32) {
      mf16_backward<P, OP, false>(lt.Ab16[0], u, 1.f, bx);
#pragma unroll
      for (int g = 0; g < KG; ++g) o[s][g] = lt.wrow[s][g] * (bx[g] * osc);
    } else {
      mf_backward<P>(lt.Ab[0], u, bx);
#pragma unroll
      for (int g = 0; g < KG; ++g) o[s][g] = lt.wrow[s][g] * bx[g];
    }
  }
  if constexpr (XF) {
    constexpr int NLX = F::NLX, GL = (N - 1) / 4, IL = (N - 1) % 4;
#pragma unroll
    for (int s = 0; s < F::SX; ++s) {
      const int l = 64 * s + lane;
      if (l < NLX) {
        xfx[(2 * wave) * NLX + l] = o[s][0][0];
        xfx[(2 * wave + 1) * NLX + l] = o[s][GL][IL];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < F::SX; ++s) {
      const int l = 64 * s + lane;
      if (l < NLX) {
        if (wave > 0) o[s][0][0] = xfx[(2 * wave - 1) * NLX + l] + o[s][0][0];
        if (wave < F::WAVES - 1) o[s][GL][IL] = o[s][GL][IL] + xfx[(2 * wave + 2) * NLX + l];
      }
    }
  }
#pragma unroll
  for (int s = 0; s < F::SX; ++s) {
    const int l = 64 * s + lane;
    if (l < F::NLX) {
      const int64_t row = e * N3 + (int64_t)l * N;  // row (j, k) = k * N + j = l
      if constexpr (N % 4 == 0) {
#pragma unroll
        for (int g = 0; g < KG; ++g) *reinterpret_cast<mf4_t *>(z + row + 4 * g) = o[s][g];
      } else {
#pragma unroll
        for (int g = 0; g < KG; ++g)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (4 * g + i < N) z[row + 4 * g + i] = o[s][g][i];
      }
    }
  }
  mf_sync();  // the next element's first pass rewrites the buffer
}

// r, rs (RS: solve on r - rs), S and lambda of the level (FP32), W = the
// grid and Dirichlet faces that give the RAS weight, z = output E-vector(s).  Each wavefront
// solves C consecutive elements, loading the next element's inputs before it
// solves the current one, so that the loads of one overlap the other's work.
template <int P, int C, bool RS, int XS, bool YS, bool XF>
__global__ __launch_bounds__(256) void k_fdm_mf32(int64_t E, int nex, int ney, int nez,
                                                  const float *__restrict__ r,
                                                  const float *__restrict__ rs,
                                                  const float *__restrict__ Sg,
                                                  const float *__restrict__ lamg,
                                                  RasW W,
                                                  float *__restrict__ z, int nv) {
  using F = Mf<P>;
  constexpr int N3 = F::N3;
  static_assert(!XF || C == 1, "x-face sums: one element per wave");
  __shared__ mf4_t lds4[F::WAVES * F::BUF / 4];
  __shared__ float xfx[XF ? 2 * F::WAVES * F::NLX : 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int vec;
  const int64_t e0 = ((int64_t)split_rhs(xcd_block(), nv, vec) * F::WAVES + wave) * C;
  // whole wave leaves; only XF waits on other waves, and then E is a multiple
  // of 4 (every wave of a workgroup is live)
  if (e0 >= E) return;
  r += (int64_t)vec * E * N3;
  if (RS) rs += (int64_t)vec * E * N3;
  z += (int64_t)vec * E * N3;
  float *buf = reinterpret_cast<float *>(lds4) + wave * F::BUF;
  // the wave reads r (and rs) only between a plane and a line below its first
  // element and as far above its last: one buffer window from there, whose
  // size the host bounds below 2 GiB
  const int64_t eb = e0 > (int64_t)nex * ney + nex + 1 ? e0 - ((int64_t)nex * ney + nex + 1) : 0;
  const int64_t wb = (E - eb) * N3 * 4;
  const uint32_t wn = wb < (int64_t)kWindowMax ? (uint32_t)wb : kWindowMax;
  const BufF32 rb(r + eb * N3, wn), rsb(RS ? rs + eb * N3 : r + eb * N3, wn);
  MfIn<P, RS, XS, YS> in[2];
  mf_load<P, RS, XS, YS>(in[0], e0, nex, ney, nez, rb, rsb, eb, Sg, lamg, W, lane);
#pragma unroll
  for (int it = 0; it < C; ++it) {
    const int64_t e = e0 + it;
    if (e >= E) break;
    if (it + 1 < C)  // (past the last element: reloads it, unused)
      mf_load<P, RS, XS, YS>(in[(it + 1) & 1], e + 1 < E ? e + 1 : e, nex, ney, nez, rb, rsb, eb, Sg,
                         lamg, W, lane);
    mf_solve<P, RS, XS, YS, XF>(in[it & 1], e, lamg, z, buf, lane, xfx, wave, Sg, W);
  }
}

// The same solve with FP16 or BF16 operands (OP), one element per wave:
// S16 = S_d / s_d as 16-bit patterns, ssc = s_d per element and direction.
// (at most 6 wavefronts per SIMD asked of the register allocator: aiming
// higher made it spill some BF16 forms at p = 7)
template <int P, bool RS, int XS, bool YS, bool XF, int OP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 6))) void k_fdm_mf16(
    int64_t E, int nex, int ney, int nez,
                                                  const float *__restrict__ r,
                                                  const float *__restrict__ rs,
                                                  const uint32_t *__restrict__ A16,
                                                  const float *__restrict__ ssc,
                                                  const float *__restrict__ lamg,
                                                  RasW W,
                                                  float *__restrict__ z, int nv) {
  using F = Mf<P>;
  constexpr int N3 = F::N3;
  __shared__ mf4_t lds4[F::WAVES * F::BUF / 4];
  __shared__ float xfx[XF ? 2 * F::WAVES * F::NLX : 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int vec;
  const int64_t e = (int64_t)split_rhs(xcd_block(), nv, vec) * F::WAVES + wave;
  if (e >= E) return;  // whole wave; XF launches only whole workgroups (E % 4 == 0)
  r += (int64_t)vec * E * N3;
  if (RS) rs += (int64_t)vec * E * N3;
  z += (int64_t)vec * E * N3;
  float *buf = reinterpret_cast<float *>(lds4) + wave * F::BUF;
  const int64_t eb = e > (int64_t)nex * ney + nex + 1 ? e - ((int64_t)nex * ney + nex + 1) : 0;
  const int64_t wb = (E - eb) * N3 * 4;
  const uint32_t wn = wb < (int64_t)kWindowMax ? (uint32_t)wb : kWindowMax;
  const BufF32 rb(r + eb * N3, wn), rsb(RS ? rs + eb * N3 : r + eb * N3, wn);
  MfIn<P, RS, XS, YS> in;
  mf_load<P, RS, XS, YS, OP>(in, e, nex, ney, nez, rb, rsb, eb, nullptr, lamg, W, lane, A16, ssc);
  mf_solve<P, RS, XS, YS, XF, OP>(in, e, lamg, z, buf, lane, xfx, wave, nullptr, W, A16, ssc);
}

static RasW ras_w(const Level &L) {
  RasW w{L.nex, L.ney, L.nez, 0, L.w32};
  for (int f = 0; f < 6; ++f) w.bcm |= (L.bc[f] ? 1 : 0) << f;
  return w;
}

template <int P, bool RS, int XS, bool YS, bool XF, int OP = kOpF32>
void mf32_launch_x(const Ctx &c, const Level &L, const float *r, const float *rs, float *z,
                   hipStream_t s, int nv) {
  using F = Mf<P>;
  if constexpr (OP != kOpF32) {
    if (XF && (L.E % F::WAVES != 0 || c.nex % F::WAVES != 0))
      fail(SEM_EINVAL, "FDM: x-face sums need whole groups of four elements along x");
    if (!L.A16 || !L.sscale) fail(SEM_EINVAL, "16-bit FDM data were not built");
    const dim3 grid((unsigned)((L.E + F::WAVES - 1) / F::WAVES * nv));
    hipLaunchKernelGGL((k_fdm_mf16<P, RS, XS, YS, XF, OP>), grid, dim3(64 * F::WAVES), 0, s, L.E,
                       c.nex, c.ney, c.nez, r, rs, L.A16, L.sscale, L.lam32, ras_w(L), z, nv);
    SEM_LAUNCH("k_fdm_mf16");
  } else {
    const int C = XF ? 1 : c.fdm_mf32_chain;
    if (XF && (L.E % F::WAVES != 0 || c.nex % F::WAVES != 0))
      fail(SEM_EINVAL, "FDM: x-face sums need whole groups of four elements along x");
    const dim3 grid((unsigned)((L.E + F::WAVES * C - 1) / (F::WAVES * C) * nv));
    const dim3 block(64 * F::WAVES);
    if constexpr (XF) {
      hipLaunchKernelGGL((k_fdm_mf32<P, 1, RS, XS, YS, true>), grid, block, 0, s, L.E, c.nex,
                         c.ney, c.nez, r, rs, L.S32, L.lam32, ras_w(L), z, nv);
    } else if (C == 2) {
      hipLaunchKernelGGL((k_fdm_mf32<P, 2, RS, XS, YS, false>), grid, block, 0, s, L.E, c.nex,
                         c.ney, c.nez, r, rs, L.S32, L.lam32, ras_w(L), z, nv);
    } else {
      hipLaunchKernelGGL((k_fdm_mf32<P, 1, RS, XS, YS, false>), grid, block, 0, s, L.E, c.nex,
                         c.ney, c.nez, r, rs, L.S32, L.lam32, ras_w(L), z, nv);
    }
    SEM_LAUNCH("k_fdm_mf32");
  }
}

// xin: 0 the inputs are assembled; 1 r, 2 rs lacks the x step of its
// gather-scatter (the kernel adds the x-neighbours' copies as it reads);
// + 4: that input lacks the y step as well (only its z step was taken);
// + 8: sum the output's x-faces inside each workgroup (assembled r, or rs
// as above), for a gather-scatter that then covers only the faces between
// workgroups
template <int P, int OP>
void mf32_launch(const Ctx &c, const Level &L, const float *r, const float *rs, float *z,
                 hipStream_t s, int nv, int xin) {
  const int which = xin & 3;
  const bool ys = (xin & 4) != 0, xf = (xin & 8) != 0;
  if (xin & ~15 || which == 3 || (ys && which == 0) || (xf && which == 1))
    fail(SEM_EINVAL, "FDM: unknown form of the deferred gather-scatter steps");
  if (which == 2 && !rs) fail(SEM_EINVAL, "FDM: no subtrahend to take the x step");
  if (rs) {
    if (which == 1) fail(SEM_EINVAL, "FDM: the x step is taken on the subtrahend only");
    if (xf) {
      if (which == 2 && ys) mf32_launch_x<P, true, 2, true, true, OP>(c, L, r, rs, z, s, nv);
      else if (which == 2) mf32_launch_x<P, true, 2, false, true, OP>(c, L, r, rs, z, s, nv);
      else mf32_launch_x<P, true, 0, false, true, OP>(c, L, r, rs, z, s, nv);
    } else {
      if (which == 2 && ys) mf32_launch_x<P, true, 2, true, false, OP>(c, L, r, rs, z, s, nv);
      else if (which == 2) mf32_launch_x<P, true, 2, false, false, OP>(c, L, r, rs, z, s, nv);
      else mf32_launch_x<P, true, 0, false, false, OP>(c, L, r, rs, z, s, nv);
    }
  } else {
    if (xf) mf32_launch_x<P, false, 0, false, true, OP>(c, L, r, rs, z, s, nv);
    else if (which == 1 && ys) mf32_launch_x<P, false, 1, true, false, OP>(c, L, r, rs, z, s, nv);
    else if (which == 1) mf32_launch_x<P, false, 1, false, false, OP>(c, L, r, rs, z, s, nv);
    else mf32_launch_x<P, false, 0, false, false, OP>(c, L, r, rs, z, s, nv);
  }
}

// Setup of L.A16 from the 16-bit factors S16 = S_d / s_d ([E][3][pb][pb]):
// for element e and direction d, the 4 QF16 lanes of the forward pairs (lane
// 4q + i, q = (kg, g): S16_d[4kg + kk][4g + i], kk < 4) and the 4 QB16 lanes of
// the backward pairs (q = (mg, g): S16_d[1 + 4g + i][4mg + kk]), four 16-bit
// patterns per lane in two words, zero past the factor.  One thread per lane
// entry.
__global__ void k_fdm_mf16_pack(int64_t E, int pb, int n, int mg, int kg, int nf, int nb,
                                const uint16_t *__restrict__ S16, uint32_t *__restrict__ A16) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int ne = nf + nb;
  if (t >= E * 3 * ne) return;
  const int64_t ed = t / ne;  // e * 3 + d
  const int j = (int)(t - ed * ne);
  const uint16_t *Sd = S16 + ed * pb * pb;
  uint32_t h[4];
  if (j < nf) {
    const int q = j >> 2, i = j & 3, k4 = q / mg, g = q % mg;
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * k4 + kk, m = 4 * g + i;
      h[kk] = k < pb && m < pb ? Sd[k * pb + m] : 0u;
    }
  } else {
    const int q = (j - nf) >> 2, i = (j - nf) & 3, m4 = q / kg, g = q % kg;
    for (int kk = 0; kk < 4; ++kk) {
      const int kn = 1 + 4 * g + i, m = 4 * m4 + kk;
      h[kk] = kn <= n && m < pb ? Sd[kn * pb + m] : 0u;
    }
  }
  A16[2 * t] = h[0] | h[1] << 16;
  A16[2 * t + 1] = h[2] | h[3] << 16;
}

struct Mf16Dims {
  int pb, n, mg, kg, nf, nb;
  explicit Mf16Dims(int p)
      : pb(p + 3), n(p + 1), mg((p + 6) / 4), kg((p + 4) / 4),
        nf(4 * ((p + 6) / 4) * ((p + 6) / 4)), nb(4 * ((p + 6) / 4) * ((p + 4) / 4)) {}
};

}  // namespace

size_t mf16_table_words(int p) {
  const Mf16Dims D(p);
  return (size_t)3 * (D.nf + D.nb) * 2;
}

void launch_fdm_mf16_pack(const Level &L, hipStream_t s) {
  if (!L.S16 || !L.A16) fail(SEM_EINVAL, "16-bit FDM data were not built");
  const Mf16Dims D(L.p);
  const int64_t n = L.E * 3 * (D.nf + D.nb);
  hipLaunchKernelGGL(k_fdm_mf16_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L.E, D.pb,
                     D.n, D.mg, D.kg, D.nf, D.nb, L.S16, L.A16);
  SEM_LAUNCH("k_fdm_mf16_pack");
}

// A box floats (a zero eigenvalue sum) only when every direction has one
// element and Neumann faces at both ends: then the 1D problem of each
// direction keeps its constant mode.
//
// A wave's reads of the box input span two planes and two lines of elements
// plus its own: their bytes must fit one buffer window.
bool fdm_mf32_supported(const Ctx &c, int p) {
  const bool floating = c.nex == 1 && c.ney == 1 && c.nez == 1 && !c.bc[0] && !c.bc[1] &&
                        !c.bc[2] && !c.bc[3] && !c.bc[4] && !c.bc[5];
  const int64_t span = 2 * ((int64_t)c.nex * c.ney + c.nex + 1) + 4;
  return p >= 2 && p <= 9 && !floating && span * (p + 1) * (p + 1) * (p + 1) * 4 < kWindowMax;
}

template <int OP>
static void mf_launch_p(const Ctx &c, const Level &L, const float *r, float *z, hipStream_t s,
                        int nv, const float *rs, int xin) {
  switch (L.p) {
    case 2: mf32_launch<2, OP>(c, L, r, rs, z, s, nv, xin); break;
    case 3: mf32_launch<3, OP>(c, L, r, rs, z, s, nv, xin); break;
    case 4: mf32_launch<4, OP>(c, L, r, rs, z, s, nv, xin); break;
    case 5: mf32_launch<5, OP>(c, L, r, rs, z, s, nv, xin); break;
    case 6: mf32_launch<6, OP>(c, L, r, rs, z, s, nv, xin); break;
    case 7: mf32_launch<7, OP>(c, L, r, rs, z, s, nv, xin); break;
    case 8: mf32_launch<8, OP>(c, L, r, rs, z, s, nv, xin); break;
    case 9: mf32_launch<9, OP>(c, L, r, rs, z, s, nv, xin); break;
    default: fail(SEM_EUNSUPPORTED, "matrix-core FDM: unsupported degree");
  }
}

void launch_fdm_mf32(const Ctx &c, const Level &L, const float *r, float *z, hipStream_t s, int nv,
                     const float *rs, int xin, int prec) {
  if (!L.S32 || !L.lam32 || !L.w32) fail(SEM_EINVAL, "FP32 FDM data were not built");
  if (prec == SEM_F16)
    mf_launch_p<kOpF16>(c, L, r, z, s, nv, rs, xin);
  else if (prec == SEM_BF16)
    mf_launch_p<kOpBF16>(c, L, r, z, s, nv, rs, xin);
  else
    mf_launch_p<kOpF32>(c, L, r, z, s, nv, rs, xin);
}

}  // namespace sem
