// Global numbering, the Boolean gather Q and direct stiffness summation QQ^T
// (Sec. 2.1: u_L = Q u; A = Q^T A_L Q).
//
// QQ^T only changes nodes held by more than one element.  The setup sorts the
// local indices of every shared node (and of every Dirichlet node, which the
// same pass zeroes) by global id, stably, so each global node becomes one
// contiguous segment of `perm`; `off[s]` is the segment start with bit 31 set
// for Dirichlet segments.  The segments are then reordered by their first
// (smallest) local index, so that consecutive threads work on neighbouring
// nodes of the same few elements.  The summation then visits each segment once, adds
// its copies in ascending local index (a fixed order: results are bitwise
// repeatable, no floating-point atomics) and writes the sum to every copy.
#include <hipcub/hipcub.hpp>

#include "sem_internal.h"

namespace sem {

struct GridInfo {
  int nex, ney, nez, p, N;
  int64_t nx, ny, nz;
  int bc[6];
};

static GridInfo grid_of(const Ctx &c, const Level &L) {
  GridInfo g;
  g.nex = c.nex; g.ney = c.ney; g.nez = c.nez; g.p = L.p; g.N = L.N;
  g.nx = (int64_t)c.nex * L.p + 1;
  g.ny = (int64_t)c.ney * L.p + 1;
  g.nz = (int64_t)c.nez * L.p + 1;
  for (int f = 0; f < 6; ++f) g.bc[f] = c.bc[f];
  return g;
}

__device__ inline void global_coords(const GridInfo &g, int64_t t, int64_t &gx, int64_t &gy,
                                     int64_t &gz) {
  int N3 = g.N * g.N * g.N;
  int64_t e = t / N3;
  int q = (int)(t - e * N3);
  int i = q % g.N, j = (q / g.N) % g.N, k = q / (g.N * g.N);
  int64_t ex = e % g.nex, ey = (e / g.nex) % g.ney, ez = e / ((int64_t)g.nex * g.ney);
  gx = ex * g.p + i;
  gy = ey * g.p + j;
  gz = ez * g.p + k;
}

__device__ inline bool is_dirichlet(const GridInfo &g, int64_t gx, int64_t gy, int64_t gz) {
  return (g.bc[0] && gx == 0) || (g.bc[1] && gx == g.nx - 1) || (g.bc[2] && gy == 0) ||
         (g.bc[3] && gy == g.ny - 1) || (g.bc[4] && gz == 0) || (g.bc[5] && gz == g.nz - 1);
}

__device__ inline bool on_interface(int64_t gc, int p, int64_t n) {
  return gc % p == 0 && gc > 0 && gc < n - 1;
}

// key = global id of shared or Dirichlet local nodes, INT32_MAX otherwise
__global__ void k_gs_keys(GridInfo g, int64_t nloc, int32_t *keys, int32_t *vals) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nloc) return;
  int64_t gx, gy, gz;
  global_coords(g, t, gx, gy, gz);
  bool shared = on_interface(gx, g.p, g.nx) || on_interface(gy, g.p, g.ny) ||
                on_interface(gz, g.p, g.nz);
  bool dir = is_dirichlet(g, gx, gy, gz);
  keys[t] = (shared || dir) ? (int32_t)((gz * g.ny + gy) * g.nx + gx) : INT32_MAX;
  vals[t] = (int32_t)t;
}

__global__ void k_gs_heads(int64_t nloc, const int32_t *skeys, int32_t *head) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nloc) return;
  int32_t k = skeys[t];
  head[t] = (k != INT32_MAX && (t == 0 || skeys[t - 1] != k)) ? 1 : 0;
}

__global__ void k_gs_offsets(GridInfo g, int64_t nloc, const int32_t *skeys, const int32_t *head,
                             const int32_t *segid, int32_t *off, int32_t *counts) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nloc) return;
  int32_t k = skeys[t];
  if (head[t]) {
    int64_t gid = k;
    int64_t gx = gid % g.nx, gy = (gid / g.nx) % g.ny, gz = gid / (g.nx * g.ny);
    bool dir = is_dirichlet(g, gx, gy, gz);
    off[segid[t]] = (int32_t)t | (dir ? (int32_t)0x80000000u : 0);
  }
  // last member of the member list: record the totals
  if (k != INT32_MAX && (t == nloc - 1 || skeys[t + 1] == INT32_MAX)) {
    counts[0] = (int32_t)(t + 1);         // members
    counts[1] = segid[t] + head[t];       // segments
  }
}

__global__ void k_gs_close(int32_t *off, const int32_t *counts) {
  off[counts[1]] = counts[0];
}

// element-major segment order: key = first (smallest) member local index
__global__ void k_seg_first(int nseg, const int32_t *perm, const int32_t *off, int32_t *key,
                            int32_t *val) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  key[s] = perm[off[s] & 0x7fffffff];
  val[s] = s;
}
__global__ void k_seg_count(int nseg, const int32_t *off, const int32_t *order, int32_t *cnt) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nseg) return;
  int s = order[t];
  cnt[t] = (off[s + 1] & 0x7fffffff) - (off[s] & 0x7fffffff);
}
__global__ void k_seg_move(int nseg, int nperm, const int32_t *perm, const int32_t *off,
                           const int32_t *order, const int32_t *start, int32_t *perm2,
                           int32_t *off2) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nseg) return;
  int s = order[t];
  int32_t a = off[s] & 0x7fffffff, b = off[s + 1] & 0x7fffffff;
  int32_t flag = off[s] & (int32_t)0x80000000u;
  for (int m = a; m < b; ++m) perm2[start[t] + (m - a)] = perm[m];
  off2[t] = start[t] | flag;
  if (t == nseg - 1) off2[nseg] = nperm;
}

template <typename T>
__global__ void k_gs(T *__restrict__ v, const int32_t *__restrict__ perm,
                     const int32_t *__restrict__ off, int nseg) {
  int s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  int32_t a = off[s];
  int32_t b = off[s + 1] & 0x7fffffff;
  bool dir = a < 0;
  a &= 0x7fffffff;
  if (dir) {
    for (int m = a; m < b; ++m) v[perm[m]] = T(0);
    return;
  }
  // at most 8 copies on a conforming hex mesh
  int32_t idx[8];
  int n = b - a;
  T sum = T(0);
  for (int m = 0; m < n && m < 8; ++m) {
    idx[m] = perm[a + m];
    sum += v[idx[m]];
  }
  for (int m = 0; m < n && m < 8; ++m) v[idx[m]] = sum;
}

// w = mask / multiplicity
__global__ void k_weights(const int32_t *__restrict__ perm, const int32_t *__restrict__ off,
                          int nseg, double *w64, float *w32) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  int32_t a = off[s];
  int32_t b = off[s + 1] & 0x7fffffff;
  bool dir = a < 0;
  a &= 0x7fffffff;
  double v = dir ? 0.0 : 1.0 / (b - a);
  for (int m = a; m < b; ++m) {
    w64[perm[m]] = v;
    if (w32) w32[perm[m]] = (float)v;
  }
}

__global__ void k_fill1(int64_t n, double *w64, float *w32) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  w64[t] = 1.0;
  if (w32) w32[t] = 1.0f;
}

__global__ void k_gather(GridInfo g, int64_t nloc, const double *__restrict__ ug,
                         double *__restrict__ ul, int64_t ug_stride) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nloc) return;
  ug += blockIdx.y * ug_stride;  // right side blockIdx.y
  ul += blockIdx.y * nloc;
  int64_t gx, gy, gz;
  global_coords(g, t, gx, gy, gz);
  ul[t] = ug[(gz * g.ny + gy) * g.nx + gx];
}

// SplitMix64 (Steele, Lea & Flood 2014) of (seed XOR gid), top 53 bits -> [-1, 1)
__device__ inline double splitmix_pm1(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

__global__ void k_start_vector(GridInfo g, int64_t nloc, uint64_t seed, const double *__restrict__ w,
                               double *__restrict__ v) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nloc) return;
  int64_t gx, gy, gz;
  global_coords(g, t, gx, gy, gz);
  uint64_t gid = (uint64_t)((gz * g.ny + gy) * g.nx + gx);
  v[t] = (w[t] != 0.0) ? splitmix_pm1(seed ^ gid) : 0.0;
}

static inline unsigned nb(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Host-only upper bound of the sort/scan temporary storage (planning must not
// touch the device): the radix sort ping-pongs keys and values through a
// second buffer pair, plus per-pass histograms; build_gather_scatter checks
// the exact requirement against this bound.
size_t gs_sort_temp_bytes(int64_t nloc) {
  return (size_t)nloc * 2 * (sizeof(int32_t) + sizeof(int32_t)) + ((size_t)8 << 20);
}

static size_t gs_sort_temp_exact(int64_t nloc) {
  size_t bytes = 0;
  SEM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (int32_t *)nullptr,
                                             (int32_t *)nullptr, (int32_t *)nullptr,
                                             (int32_t *)nullptr, (int)nloc));
  size_t scan = 0;
  SEM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (int32_t *)nullptr, (int32_t *)nullptr,
                                           (int)nloc));
  return bytes > scan ? bytes : scan;
}

void build_gather_scatter(const Ctx &c, Level &L, Arena &scratch, hipStream_t s) {
  GridInfo g = grid_of(c, L);
  int64_t n = L.nloc;
  int32_t *keys = scratch.take<int32_t>(n);
  int32_t *vals = scratch.take<int32_t>(n);
  int32_t *skeys = scratch.take<int32_t>(n);
  int32_t *head = scratch.take<int32_t>(n);
  int32_t *segid = scratch.take<int32_t>(n);
  int32_t *counts = scratch.take<int32_t>(4);
  size_t tb = gs_sort_temp_exact(n);
  if (tb > gs_sort_temp_bytes(n)) fail(SEM_EHIP, "sort scratch larger than planned");
  char *tmp = scratch.take<char>(tb);
  hipLaunchKernelGGL(k_gs_keys, dim3(nb(n, 256)), dim3(256), 0, s, g, n, keys, vals);
  SEM_LAUNCH("k_gs_keys");
  size_t tb2 = tb;
  SEM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb2, keys, skeys, vals, L.perm, (int)n, 0,
                                             32, s));
  hipLaunchKernelGGL(k_gs_heads, dim3(nb(n, 256)), dim3(256), 0, s, n, skeys, head);
  SEM_LAUNCH("k_gs_heads");
  tb2 = tb;
  SEM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb2, head, segid, (int)n, s));
  SEM_HIP(hipMemsetAsync(counts, 0, 4 * sizeof(int32_t), s));
  hipLaunchKernelGGL(k_gs_offsets, dim3(nb(n, 256)), dim3(256), 0, s, g, n, skeys, head, segid,
                     L.off, counts);
  SEM_LAUNCH("k_gs_offsets");
  hipLaunchKernelGGL(k_gs_close, dim3(1), dim3(1), 0, s, L.off, counts);
  SEM_LAUNCH("k_gs_close");
  int32_t h[4];
  SEM_HIP(hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  L.nperm = h[0];
  L.nseg = h[1];
  if (L.nseg == 0) return;
  // reorder the segments element-major (by their first copy) so that a
  // wavefront's segments touch neighbouring memory; members stay sorted
  const int ns = L.nseg;
  int32_t *order = head, *cnt = segid, *start = keys;
  int32_t *perm2 = scratch.take<int32_t>(n);
  int32_t *off2 = scratch.take<int32_t>(n + 1);
  int32_t *k2 = scratch.take<int32_t>(n);
  hipLaunchKernelGGL(k_seg_first, dim3(nb(ns, 256)), dim3(256), 0, s, ns, L.perm, L.off, k2, vals);
  SEM_LAUNCH("k_seg_first");
  tb2 = tb;
  SEM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb2, k2, skeys, vals, order, ns, 0, 32, s));
  hipLaunchKernelGGL(k_seg_count, dim3(nb(ns, 256)), dim3(256), 0, s, ns, L.off, order, cnt);
  SEM_LAUNCH("k_seg_count");
  tb2 = tb;
  SEM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb2, cnt, start, ns, s));
  hipLaunchKernelGGL(k_seg_move, dim3(nb(ns, 256)), dim3(256), 0, s, ns, L.nperm, L.perm, L.off,
                     order, start, perm2, off2);
  SEM_LAUNCH("k_seg_move");
  SEM_HIP(hipMemcpyAsync(L.perm, perm2, (size_t)L.nperm * sizeof(int32_t),
                         hipMemcpyDeviceToDevice, s));
  SEM_HIP(hipMemcpyAsync(L.off, off2, (size_t)(ns + 1) * sizeof(int32_t),
                         hipMemcpyDeviceToDevice, s));
  SEM_HIP(hipStreamSynchronize(s));
}

// The same summation on the structured element grid, one direction per pass:
// the copies of a node on the faces normal to direction D of two neighbouring
// elements are summed pairwise, and the Dirichlet faces of that direction are
// zeroed.  After the x, y and z passes every copy holds the sum of all copies
// (2, 4 or 8) and Dirichlet nodes are 0; each pairwise sum is symmetric, so
// the copies agree bit for bit.  No index arrays: thread (e, line) touches the
// line's two face nodes and the neighbour's facing node.
struct GsGrid {
  int nex, ney, nez, p, N;
  int bc[6];
};

template <typename T, int D>
__global__ void k_gs_dir(T *__restrict__ v, GsGrid g, int64_t E) {
  const int64_t t = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  const int N = g.N, N2 = N * N;
  if (t >= E * N2) return;
  v += blockIdx.y * E * N2 * N;  // right side blockIdx.y
  const unsigned ut = (unsigned)t;  // E * N^2 < 2^31
  const int64_t e = ut / (unsigned)N2;
  const int rem = (int)(ut - (unsigned)e * (unsigned)N2);
  int64_t ex, ey, ez;
  elem_coords(e, g.nex, g.ney, ex, ey, ez);
  const int64_t N3 = (int64_t)N2 * N;
  int64_t lo, hi, step;
  int64_t pos, cnt;
  int blo, bhi;
  if (D == 0) {  // line along i through (j, k) = rem
    lo = e * N3 + (int64_t)rem * N;
    hi = lo + g.p;
    step = N3;
    pos = ex; cnt = g.nex; blo = g.bc[0]; bhi = g.bc[1];
  } else if (D == 1) {  // line along j through (i, k)
    const int k = rem / N, i = rem - k * N;
    lo = e * N3 + (int64_t)k * N2 + i;
    hi = lo + (int64_t)g.p * N;
    step = (int64_t)g.nex * N3;
    pos = ey; cnt = g.ney; blo = g.bc[2]; bhi = g.bc[3];
  } else {  // line along k through (i, j)
    lo = e * N3 + rem;
    hi = lo + (int64_t)g.p * N2;
    step = (int64_t)g.nex * g.ney * N3;
    pos = ez; cnt = g.nez; blo = g.bc[4]; bhi = g.bc[5];
  }
  if (pos + 1 < cnt) {
    const T sum = v[hi] + v[lo + step];
    v[hi] = sum;
    v[lo + step] = sum;
  }
  if (pos == 0 && blo) v[lo] = T(0);
  if (pos == cnt - 1 && bhi) v[hi] = T(0);
}

// The x pass when the faces inside each group of 4 consecutive elements along x
// are summed already: thread (group q, line) sums the face between the group's
// last element and the next group's first, and zeroes the Dirichlet x-faces of
// the row ends (the low face of the group's first element, the high face of
// its last).  Requires nex to be a multiple of 4.
template <typename T>
__global__ void k_gs_xb(T *__restrict__ v, GsGrid g, int64_t E) {
  const int64_t t = xcd_block() * (int64_t)blockDim.x + threadIdx.x;
  const int N = g.N, N2 = N * N;
  const int64_t groups = E / 4;
  if (t >= groups * N2) return;
  v += blockIdx.y * E * N2 * N;  // right side blockIdx.y
  const unsigned ut = (unsigned)t;
  const int64_t q = ut / (unsigned)N2;
  const int rem = (int)(ut - (unsigned)q * (unsigned)N2);
  const int64_t N3 = (int64_t)N2 * N;
  const int64_t e0 = 4 * q, e3 = e0 + 3;
  const int64_t ex0 = e0 % g.nex, ex3 = ex0 + 3;
  const int64_t line = (int64_t)rem * N;
  if (g.bc[0] && ex0 == 0) v[e0 * N3 + line] = T(0);
  const int64_t hi = e3 * N3 + line + g.p;
  if (ex3 + 1 < g.nex) {
    const int64_t lo = (e3 + 1) * N3 + line;
    const T sum = v[hi] + v[lo];
    v[hi] = sum;
    v[lo] = sum;
  } else if (g.bc[1]) {
    v[hi] = T(0);
  }
}

// The y and z passes in one launch, with the same sums in the same order.
// Thread sets (i fastest in each):
//   Y: rows of a y-face with k = 1..p-1 (the z pass never touches them),
//   Z: rows of a z-face with j = 1..p-1 (the y pass never touches them),
//   E: the x-lines where y- and z-faces meet (j, k in {0, p}): up to four
//      copies; the y step (pair sum, or the Dirichlet zero / the value itself
//      at a y boundary) is taken on each z side, then the z step on the
//      results, and the total goes to every copy: (a + b) + (c + d), as the
//      two passes compute it.
// Every face node belongs to exactly one thread; the whole vector is read
// once instead of once per pass.  Measured at 32^3, p = 7: 10 % faster than the
// two passes in FP64, 7 % slower in FP32; used for FP64 by default.
template <typename T>
__global__ void k_gs_yz(T *__restrict__ v, GsGrid g, int64_t E, int64_t ny_t, int64_t nz_t,
                        int64_t ne_t) {
  // thread counts and element indices stay below 2^31 (E N^2 < 2^31): 32-bit
  // unsigned index arithmetic
  const unsigned t0 = xcd_block() * blockDim.x + threadIdx.x;
  const unsigned nyz = (unsigned)(ny_t + nz_t);
  if (t0 >= nyz + (unsigned)ne_t) return;
  const unsigned N = (unsigned)g.N, p = (unsigned)g.p, N2 = N * N;
  const unsigned nex = (unsigned)g.nex, ney = (unsigned)g.ney, nez = (unsigned)g.nez;
  const int64_t N3 = (int64_t)N2 * N;
  v += blockIdx.y * E * N3;  // right side blockIdx.y
  auto elem = [&](unsigned ex, unsigned ey, unsigned ez) {
    return (int64_t)((ez * ney + ey) * nex + ex);
  };
  if (t0 < nyz) {  // a y-face row (k interior) or a z-face row (j interior)
    const bool yf = t0 < (unsigned)ny_t;
    unsigned t = yf ? t0 : t0 - (unsigned)ny_t;
    const unsigned i = t % N;
    t /= N;
    const unsigned m = 1 + t % (p - 1);  // k (y-face) or j (z-face)
    t /= p - 1;
    const unsigned ex = t % nex;
    t /= nex;
    const unsigned cnt = yf ? ney : nez;
    const unsigned gf = t % (cnt + 1), other = t / (cnt + 1);  // face index; ez (y) or ey (z)
    const bool has_lo = gf >= 1, has_up = gf < cnt;
    const int64_t lo_e = has_lo ? (yf ? elem(ex, gf - 1, other) : elem(ex, other, gf - 1)) : 0;
    const int64_t up_e = has_up ? (yf ? elem(ex, gf, other) : elem(ex, other, gf)) : 0;
    // lower copy: the element's p-face; upper copy: the 0-face
    const unsigned lo = yf ? m * N2 + p * N + i : p * N2 + m * N + i;
    const unsigned up = yf ? m * N2 + i : m * N + i;
    const int blo = yf ? g.bc[2] : g.bc[4], bhi = yf ? g.bc[3] : g.bc[5];
    T *const a = v + lo_e * N3 + lo;
    T *const b = v + up_e * N3 + up;
    if (has_lo && has_up) {
      const T sum = *a + *b;
      *a = sum;
      *b = sum;
    } else if (has_lo) {
      if (bhi) *a = T(0);
    } else if (has_up) {
      if (blo) *b = T(0);
    }
    return;
  }
  // an x-line where y- and z-faces meet
  unsigned t = t0 - nyz;
  const unsigned i = t % N;
  t /= N;
  const unsigned ex = t % nex;
  t /= nex;
  const unsigned gy = t % (ney + 1), gz = t / (ney + 1);
  int64_t idx[2][2];  // [z side][y side], -1 when absent
#pragma unroll
  for (int zs = 0; zs < 2; ++zs)
#pragma unroll
    for (int ys = 0; ys < 2; ++ys) {
      const bool in = (ys ? gy < ney : gy >= 1) && (zs ? gz < nez : gz >= 1);
      idx[zs][ys] = in ? elem(ex, gy - 1 + ys, gz - 1 + zs) * N3 + (zs ? 0 : p) * N2 +
                             (ys ? 0 : p) * N + i
                       : -1;
    }
  T zv[2];
  bool zin[2];
#pragma unroll
  for (int zs = 0; zs < 2; ++zs) {
    const int64_t a = idx[zs][0], b = idx[zs][1];
    zin[zs] = a >= 0 || b >= 0;
    if (a >= 0 && b >= 0)
      zv[zs] = v[a] + v[b];
    else if (a >= 0)
      zv[zs] = g.bc[3] ? T(0) : v[a];
    else if (b >= 0)
      zv[zs] = g.bc[2] ? T(0) : v[b];
    else
      zv[zs] = T(0);
  }
  T tot;
  if (zin[0] && zin[1])
    tot = zv[0] + zv[1];
  else if (zin[0])
    tot = g.bc[5] ? T(0) : zv[0];
  else
    tot = g.bc[4] ? T(0) : zv[1];
#pragma unroll
  for (int zs = 0; zs < 2; ++zs)
#pragma unroll
    for (int ys = 0; ys < 2; ++ys)
      if (idx[zs][ys] >= 0) v[idx[zs][ys]] = tot;
}

template <typename T>
void launch_gs(const Level &L, T *v, hipStream_t s, int nv, bool x_in_blocks, bool skip_x,
               bool skip_y) {
  if (x_in_blocks && (!L.gs_struct || L.nex % 4 != 0))
    fail(SEM_EINVAL, "gather-scatter: block x-faces need the direction passes and nex % 4 == 0");
  if ((skip_x || skip_y) && !L.gs_struct)
    fail(SEM_EINVAL, "gather-scatter: skipping a pass needs the direction passes");
  if (L.gs_struct) {
    GsGrid g;
    g.nex = L.nex; g.ney = L.ney; g.nez = L.nez; g.p = L.p; g.N = L.N;
    for (int f = 0; f < 6; ++f) g.bc[f] = L.bc[f];
    const dim3 grid(nb(L.E * L.N * L.N, 256), (unsigned)nv);
    if (skip_x) {
      // the consumer takes the x step (the passes commute up to rounding)
    } else if (x_in_blocks) {
      const dim3 gx(nb(L.E / 4 * L.N * L.N, 256), (unsigned)nv);
      hipLaunchKernelGGL((k_gs_xb<T>), gx, dim3(256), 0, s, v, g, L.E);
      SEM_LAUNCH("k_gs_xb");
    } else {
      hipLaunchKernelGGL((k_gs_dir<T, 0>), dim3(grid), dim3(256), 0, s, v, g, L.E);
      SEM_LAUNCH("k_gs_dir");
    }
    if (skip_y) {  // z pass only (the consumer takes the y step)
      hipLaunchKernelGGL((k_gs_dir<T, 2>), dim3(grid), dim3(256), 0, s, v, g, L.E);
      SEM_LAUNCH("k_gs_dir");
      return;
    }
    const bool yz = L.gs_yz == 1 || (L.gs_yz < 0 && sizeof(T) == 8);
    if (yz && L.p >= 2) {
      const int64_t ny_t = (int64_t)L.nex * (L.ney + 1) * L.nez * (L.p - 1) * L.N;
      const int64_t nz_t = (int64_t)L.nex * L.ney * (L.nez + 1) * (L.p - 1) * L.N;
      const int64_t ne_t = (int64_t)L.nex * (L.ney + 1) * (L.nez + 1) * L.N;
      const dim3 gyz(nb(ny_t + nz_t + ne_t, 256), (unsigned)nv);
      hipLaunchKernelGGL((k_gs_yz<T>), gyz, dim3(256), 0, s, v, g, L.E, ny_t, nz_t, ne_t);
      SEM_LAUNCH("k_gs_yz");
      return;
    }
    hipLaunchKernelGGL((k_gs_dir<T, 1>), dim3(grid), dim3(256), 0, s, v, g, L.E);
    SEM_LAUNCH("k_gs_dir");
    hipLaunchKernelGGL((k_gs_dir<T, 2>), dim3(grid), dim3(256), 0, s, v, g, L.E);
    SEM_LAUNCH("k_gs_dir");
    return;
  }
  if (L.nseg == 0) return;
  for (int k = 0; k < nv; ++k) {
    hipLaunchKernelGGL(k_gs<T>, dim3(nb(L.nseg, 256)), dim3(256), 0, s, v + k * L.nloc, L.perm,
                       L.off, L.nseg);
    SEM_LAUNCH("k_gs");
  }
}
template void launch_gs<double>(const Level &, double *, hipStream_t, int, bool, bool, bool);
template void launch_gs<float>(const Level &, float *, hipStream_t, int, bool, bool, bool);

void launch_weights(const Level &L, hipStream_t s) {
  hipLaunchKernelGGL(k_fill1, dim3(nb(L.nloc, 256)), dim3(256), 0, s, L.nloc, L.w64, L.w32);
  SEM_LAUNCH("k_fill1");
  if (L.nseg == 0) return;
  hipLaunchKernelGGL(k_weights, dim3(nb(L.nseg, 256)), dim3(256), 0, s, L.perm, L.off, L.nseg,
                     L.w64, L.w32);
  SEM_LAUNCH("k_weights");
}

void launch_gather(const Ctx &c, const Level &L, const double *ug, double *ul, hipStream_t s,
                   int nv, int64_t ug_stride) {
  GridInfo g = grid_of(c, L);
  hipLaunchKernelGGL(k_gather, dim3(nb(L.nloc, 256), (unsigned)nv), dim3(256), 0, s, g, L.nloc,
                     ug, ul, ug_stride);
  SEM_LAUNCH("k_gather");
}

void launch_start_vector(const Ctx &c, const Level &L, uint64_t seed, double *v, hipStream_t s) {
  GridInfo g = grid_of(c, L);
  hipLaunchKernelGGL(k_start_vector, dim3(nb(L.nloc, 256)), dim3(256), 0, s, g, L.nloc, seed,
                     L.w64, v);
  SEM_LAUNCH("k_start_vector");
}

}  // namespace sem
