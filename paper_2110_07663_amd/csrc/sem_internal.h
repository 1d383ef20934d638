// Internal declarations of the SE Poisson library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <utility>
#include <initializer_list>
#include <vector>

#include "sem.h"

namespace sem {

// ---------------------------------------------------------------------------
// errors: internal code throws sem::Error; the ABI layer converts it to a status
struct Error {
  sem_status status;
  std::string msg;
};

[[noreturn]] void fail(sem_status st, const std::string &msg);
void set_last_error(const std::string &msg);
void check_hip(hipError_t e, const char *what, const char *file, int line);
#define SEM_HIP(call) ::sem::check_hip((call), #call, __FILE__, __LINE__)
#define SEM_LAUNCH(what) ::sem::check_hip(hipGetLastError(), what, __FILE__, __LINE__)

constexpr int kMaxP = 10;      // highest supported polynomial degree
constexpr int kMaxLevels = 8;
constexpr int kMaxArnoldi = 16;

// Element coordinates in the structured element grid (element counts stay
// below 2^31, so 32-bit unsigned division suffices)
__device__ inline void elem_coords(int64_t e, int nex, int ney, int64_t &ex, int64_t &ey,
                                   int64_t &ez) {
  const unsigned ue = (unsigned)e, q = ue / (unsigned)nex;
  ex = ue - q * (unsigned)nex;
  ey = q % (unsigned)ney;
  ez = q / (unsigned)ney;
}

// The weight of a level's local node, mask / multiplicity, on the structured
// element grid: a product over the three directions of 1 (inside the
// element, or on a Neumann face of the domain), 1/2 (on a face shared with a
// neighbour) and 0 (on a Dirichlet face), exact in floating point and equal
// to the assembled weight.  Per-direction factor of index i (0..N-1) in the
// element at grid position c of n; bcm bit f (f + 1) set when the low (high)
// domain face of the direction is Dirichlet.
__device__ inline float node_w1(int i, int N, int64_t c, int n, int bcm, int f) {
  if (i == 0) return c > 0 ? 0.5f : ((bcm >> f) & 1 ? 0.f : 1.f);
  if (i == N - 1) return c + 1 < n ? 0.5f : ((bcm >> (f + 1)) & 1 ? 0.f : 1.f);
  return 1.f;
}
// Workgroups are dispatched to the device's 8 XCDs round-robin (block b runs on
// XCD b % 8), and each XCD has its own L2.  Kernels whose blocks read their
// neighbours' data (gather-scatter segments, Schwarz boxes) renumber their
// blocks so that each XCD walks one contiguous range of logical blocks; the
// neighbours of a block then live in the same L2.  A bijection of [0, gridDim.x).
__device__ inline unsigned xcd_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned x = b & 7u, q = b >> 3, per = nb >> 3, rem = nb & 7u;
  return x * per + (x < rem ? x : rem) + q;
}
// Launches over nv right sides (vectors nloc apart) run nv logical blocks per
// element group, consecutive so that they share an XCD and its L2: logical
// block q is element group q / nv of right side q % nv.
__device__ inline unsigned split_rhs(unsigned q, int nv, int &vec) {
  if (nv == 1) {
    vec = 0;
    return q;
  }
  vec = (int)(q % (unsigned)nv);
  return q / (unsigned)nv;
}
constexpr int kMaxRestart = 64;

// ---------------------------------------------------------------------------
// bump allocator over the caller's workspace; with base == nullptr it only
// counts bytes (planning pass), so plan and setup walk the same sequence
struct Arena {
  char *base = nullptr;
  size_t off = 0, cap = 0;
  template <typename T>
  T *take(size_t n) {
    off = (off + 255) & ~size_t(255);
    size_t at = off;
    off += n * sizeof(T);
    if (!base) return nullptr;
    if (off > cap) fail(SEM_EWORKSPACE, "workspace exhausted while carving buffers");
    return reinterpret_cast<T *>(base + at);
  }
};

// ---------------------------------------------------------------------------
// one multigrid level
struct Level {
  int p = 0, N = 0, N3 = 0, pb = 0;  // pb = p + 3 (extended Schwarz box)
  int64_t E = 0, nloc = 0, nglob = 0;
  int nseg = 0, nperm = 0;           // gather-scatter segments and member count
  bool fine = false, coarse = false;
  bool lowp = false;                 // level kept in FP32 for the smoother
  int ax_variant = 2;                // Ax kernel shape at p = 7 (0 generic, 1 one wave/element, 2 non-temporal)
  // structured element grid (x fastest) and boundary conditions, for the
  // direction-by-direction gather-scatter
  int nex = 0, ney = 0, nez = 0;
  int bc[6] = {0, 0, 0, 0, 0, 0};
  bool gs_struct = true;             // false: the sorted-numbering segments (perm/off)
  bool xfuse = true;                 // the p = 7 Ax sums x-faces inside its workgroups
  int gs_yz = -1;                    // y and z passes in one launch: 1 yes, 0 no, -1 FP64 only
  bool xdefer = true;                // Chebyshev updates may take the x step of S's gather-scatter
  bool ydefer = true;                // ... and its y step
  double *dotpart = nullptr;         // [E] element shares of (p, Ap) (finest level)

  // 1D operators (device): GLL nodes/weights, derivative matrix D[i][j] = h_j'(xi_i)
  double *xi = nullptr, *wq = nullptr, *D64 = nullptr;
  float *D32 = nullptr;
  // interpolation from the next coarser level: J[N][Nc], J[i][j] = h^c_j(xi_i)
  double *J64 = nullptr;
  float *J32 = nullptr;

  // geometry (device)
  double *X = nullptr;     // [3][nloc] node coordinates
  double *G64 = nullptr;   // [E][6][N3] (rr, rs, rt, ss, st, tt)
  float *G32 = nullptr;    // FP32 copy for the smoother
  uint32_t *G16 = nullptr;  // FP16 pairs (G0,G1), (G2,G3), (G4,G5): [E][3][N^3], scaled per element
  float *gscale = nullptr;  // [E]: the power of two that undoes an element's G16 scaling
  double *BL = nullptr;    // [nloc] diagonal mass (finest level)
  double *w64 = nullptr;   // [nloc] mask / multiplicity (dot weight, RAS weight)
  float *w32 = nullptr;
  double *dinv64 = nullptr;  // [nloc] Jacobi: 1/diag(A), 0 on Dirichlet nodes
  float *dinv32 = nullptr;

  // gather-scatter: perm[] = local indices of shared/Dirichlet nodes sorted by
  // global id; off[s] = start of segment s, bit 31 set for Dirichlet segments
  int32_t *perm = nullptr, *off = nullptr;

  // FDM (Schwarz) data: S[E][3][pb][pb] (column a of direction d at [e][d][.][a]),
  // lam[E][3][pb] (+inf marks a decoupled node)
  double *S64 = nullptr, *lam64 = nullptr;
  float *S32 = nullptr, *lam32 = nullptr;
  uint16_t *S16 = nullptr;  // S / s_d in BF16 or FP16 bit patterns (MFMA path)
  float *sscale = nullptr;  // [E][3] s_d = max |S_d|
  uint32_t *A16 = nullptr;  // the 16-bit line kernel's A operands of S16, in lane order
  double *boxlen = nullptr; // [E][3]
  double *box64 = nullptr;  // [E][pb^3] ASM local-solve outputs before the overlap sum
  float *box32 = nullptr;

  // Chebyshev parameters
  double lam_tilde = 0, lmin = 0, lmax = 0;
  int K = 0;

  // work E-vectors of this level: FP64 set and FP32 set
  double *d_b = nullptr, *d_x = nullptr, *d_r = nullptr, *d_d = nullptr, *d_w = nullptr,
         *d_t = nullptr;
  float *f_b = nullptr, *f_x = nullptr, *f_r = nullptr, *f_d = nullptr, *f_w = nullptr,
        *f_t = nullptr;
};

// device-resident scalars of the coarse PCG and of reductions
struct DevScalars {
  double rz, pq, alpha, beta, rr, rr0, tol2;
  int done, iters, maxit;
  int aborted;  // set when a grid barrier of the persistent solve timed out
};

// scalars of the coarse-grid CG (device resident)
struct CoarseScalars {
  double gamma, gamma_old, delta, alpha, beta, rr, rr0, tol2;
  int done, iters, maxit;
  int aborted;  // set when a grid barrier of the persistent solve timed out
};

// assembled p = 1 coarse operator and its CG state (buffers in the workspace)
struct CoarseSolver {
  int64_t n = 0;                   // global nodes of the coarsest level
  double *St = nullptr;            // [27][n] stencil values
  double *dinv = nullptr;          // [n]
  double *Ae = nullptr;            // [E][8][8] element matrices (setup only)
  double *b = nullptr, *x = nullptr, *r = nullptr, *u = nullptr, *w = nullptr, *p = nullptr,
         *s = nullptr;
  double *r2 = nullptr, *w2 = nullptr, *s2 = nullptr;  // alternate copies of r, w, s
  double *partials = nullptr;      // [2][blocks][4]
  unsigned *counter = nullptr;     // [64]: [0] last-block counter, [32] grid-barrier arrivals
  CoarseScalars *sc = nullptr;
  int chunk = 16;                  // iterations per recorded graph (even)
  bool use_graph = true;
  bool persistent = false;         // whole solve in one cooperative launch
  // exact block-tridiagonal solve (coarse_direct.hip): G, H, J blocks, work vector
  bool direct = false;
  double *dG = nullptr, *dH = nullptr, *dJ = nullptr, *dy = nullptr;
  float *fG = nullptr, *fH = nullptr, *fJ = nullptr;  // FP32 copies read by the sweeps (FP32 smoother)
  int *dflag = nullptr;
  hipStream_t cap = nullptr;       // private capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// HIP-event timing of finest-level kernels (sem_profile)
struct Profiler {
  bool on = false;
  unsigned kinds = ~0u;  // bit k: record class k
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;  // events of the current session
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  size_t used = 0;
  size_t begin(int kind, hipStream_t s);
  void end(size_t rec, hipStream_t s);
  void reset();
  ~Profiler();
};

struct Ctx {
  int nex = 0, ney = 0, nez = 0;
  Profiler *prof = nullptr;
  int bc[6] = {0, 0, 0, 0, 0, 0};
  sem_opts opts{};
  int nlev = 0;
  Level lev[kMaxLevels];
  bool lowp = false;  // smoother levels in FP32

  // reductions
  double *partials = nullptr;   // [kRedBlocks][8]
  unsigned *counter = nullptr;  // last-block counter
  double *dres = nullptr;       // [64] reduction results
  DevScalars *dsc = nullptr;
  double *hres = nullptr;       // host copy (pinned)

  // outer Krylov vectors (FP64, finest level)
  double *kr = nullptr, *kz = nullptr, *kzold = nullptr, *kp = nullptr, *kq = nullptr,
         *kx = nullptr;
  float *fzo = nullptr;  // mixed path: the previous FP32 preconditioned residual (nvmax x nloc)
  double *gV = nullptr, *gZ = nullptr;  // FGMRES bases [(m+1)][nloc], [m][nloc]
  // A-conjugate projection onto prior solutions: X [proj_max][nloc] (A-orthonormal),
  // AX = A X, and two work vectors; nproj basis vectors in use
  double *projX = nullptr, *projAX = nullptr, *projW = nullptr, *projAW = nullptr;
  int nproj = 0;
  // coarse PCG vectors (FP64, coarsest level)
  double *cx = nullptr, *cr = nullptr, *cz = nullptr, *cp = nullptr, *cq = nullptr;
  int last_coarse_iters = 0;
  // graph capture of whole iterations (batched solves): no host synchronisation
  // may be enqueued, so the coarse solve runs a fixed number of iterations
  bool capturing = false;
  int capture_coarse_iters = 0;
  // batched-solve lanes: per right side r, z, z_old, p, q (FP64) and scalars
  int nlanes = 0;
  double *lanev = nullptr;           // [5][nlanes][nloc]: r, z, z_old, p, q of every lane
  void *lanes = nullptr;
  double *lpartials = nullptr;       // [nlanes][kRedBlocks][8] lane reductions
  // level work vectors (and the coarse solve's vectors) hold nvmax right sides,
  // so the lanes of a batched solve share one V-cycle (nvmax = nlanes), else 1
  int nvmax = 1;
  CoarseSolver coarse_store;
  CoarseSolver *cs = nullptr;      // set when the coarsest level is p = 1 (assembled solve)
  // Arnoldi basis (FP64, largest level)
  double *av = nullptr;
  int fdm_prec = SEM_F32;
  bool fdm_lines = true;  // line-organised VALU FDM kernel for pbar^2 > 64
  bool fdm_group = true;  // p <= 3: several elements' boxes per workgroup of 256 threads
  bool fdm_mfma1 = false; // first matrix-core FDM form (LDS FP32 box) instead of the second
  bool fdm_mf32 = true;   // FP32 RAS local solves on the matrix cores (fdm_mf32.hip)
  int fdm_mf32_chain = 1; // elements per wavefront there (1 or 2), next one's loads ahead
  bool fdm_mf16 = true;   // FP16 / BF16 RAS operands in that kernel's 4x4x4 form
  bool fdm_xstep = true;  // that kernel takes the x step of A's gather-scatter as it reads
  bool fdm_ystep = true;  // ... and the y step as well (A's gather-scatter takes only z)
  bool fdm_xfaces = true;  // ... and sums its output's x-faces inside each workgroup
  bool coarse_sum = true;  // the assembled coarse solve sums the restricted copies itself
};

// ---------------------------------------------------------------------------
// kernel launchers (each enqueues on `s`)
constexpr int kRedBlocks = 1024;

// basis.hip
void launch_gll(int p, double *xi, double *w, hipStream_t s);
void launch_dmat(int p, const double *xi, double *D, float *D32, hipStream_t s);
void launch_interp(int pc, int pf, const double *xic, const double *xif, double *J, float *J32,
                   hipStream_t s);

// geom.hip
void launch_level_coords(const Ctx &c, const double *xyz_in, int p_geom, const double *Jg,
                         Level &L, hipStream_t s);
void launch_geom(const Ctx &c, Level &L, int *bad_flag, hipStream_t s);
void launch_geom16(Level &L, hipStream_t s);  // FP16 copy of G for the FP32 smoother (p = 7)
void launch_boxlen(const Ctx &c, Level &L, hipStream_t s);
void launch_rhs(const Level &L, const double *f, double *b, hipStream_t s);

// numbering.hip
size_t gs_sort_temp_bytes(int64_t nloc);
void build_gather_scatter(const Ctx &c, Level &L, Arena &scratch, hipStream_t s);
void launch_gather(const Ctx &c, const Level &L, const double *ug, double *ul, hipStream_t s,
                   int nv = 1, int64_t ug_stride = 0);
// nv > 1: nv vectors nloc apart (several right sides of one problem)
// x_in_blocks: the x-faces inside each group of 4 elements along x are summed
// already (Ax with xf); only the faces between groups and the Dirichlet x-faces
// remain for the x pass
template <typename T>
void launch_gs(const Level &L, T *v, hipStream_t s, int nv = 1, bool x_in_blocks = false,
               bool skip_x = false, bool skip_y = false);  // skip: leave that pass out
void launch_weights(const Level &L, hipStream_t s);
void launch_start_vector(const Ctx &c, const Level &L, uint64_t seed, double *v, hipStream_t s);

// ax.hip
// xf: also sum the x-faces shared inside each workgroup (see ax_sums_x_faces);
// the following launch_gs must then be told (x_in_blocks)
template <typename T>
void launch_ax(const Level &L, const T *u, T *v, hipStream_t s, int nv = 1, bool xf = false,
               double *dotp = nullptr);
// the FP64 Ax of this level can write each element's share of (u, Au) (dotp[e])
bool ax_forms_dot(const Level &L, int nv);
// out = sum of part[0..n) in a fixed order
void launch_sum_partials(int64_t n, const double *part, double *out, hipStream_t s);
bool ax_sums_x_faces(const Level &L);
void launch_diag(const Level &L, double *d, hipStream_t s);

// blas.hip
template <typename T>
void launch_scale(int64_t n, const T *w, const T *x, T *y, hipStream_t s);  // y = w.*x
void launch_copy_cvt_d2f(int64_t n, const double *x, float *y, hipStream_t s);
void launch_copy_cvt_f2d(int64_t n, const float *x, double *y, hipStream_t s);
template <typename T>
void launch_axpby(int64_t n, T a, const T *x, T b, T *y, hipStream_t s);  // y = a x + b y
template <typename T>
void launch_sub(int64_t n, const T *a, const T *b, T *y, hipStream_t s);  // y = a - b
// The x step of the gather-scatter left to the Chebyshev update that reads t
// (the y and z passes done): each copy on an x-face adds its neighbour's copy
// as it reads, (p-face + 0-face), and the Dirichlet x-faces read as zero.
// on = false: t is assembled already.
struct XDefer {
  bool on = false;
  int nex = 0, N = 0, bc0 = 0, bc1 = 0;
  int64_t nloc = 0;  // right sides nloc apart
  bool y = false;    // the y step too (the gather-scatter ran its z pass only)
  int ney = 0, bc2 = 0, bc3 = 0;
};
// whether launch_cheb_* can take the x step for these vectors (16-byte
// vectors that do not straddle the element rows)
template <typename T>
bool cheb_can_defer_x(int N, int64_t n, std::initializer_list<const void *> ps);
// x_zero: x is zero on entry (not read)
template <typename T>
void launch_cheb_update(int64_t n, T *x, T *r, T *d, const T *t, T a, T c, hipStream_t s,
                        bool x_zero = false, const XDefer &xd = XDefer());
template <typename T>
void launch_cheb_last(int64_t n, T *x, const T *r, const T *d, const T *t, T a, T c,
                      hipStream_t s, bool x_zero = false,
                      const XDefer &xd = XDefer());  // x += d + (a d + c (r - t))
// first pass from r_0 and t = S A r_0 (d_0 = r_0 / theta formed inside)
template <typename T>
void launch_cheb_first(int64_t n, T *x, T *r, T *d, const T *t, T inv_theta, T a, T c,
                       bool x_zero, bool last, hipStream_t s, const XDefer &xd = XDefer());
void launch_jacobi_inv(int64_t n, const double *diag, const double *w, double *dinv, float *dinv32,
                       hipStream_t s);
// weighted dots: out[j] = sum_i w_i a_j(i) b_j(i), j < nd <= 4 (fixed-order reduction)
// (w32: an FP32 copy of the weights, used when given; the weights are exact in FP32)
// (rf: also store the new r in FP32 there, when given)
// (alpha = rz / pq from the device, 0 when pq <= 0)
// (xq.on: q comes without the x and y steps of its gather-scatter, taken as read)
void launch_fcg_xr(const Ctx &c, int64_t n, const double *rz, const double *pq, const double *w,
                   const double *p, const double *q, double *x, double *r, double *out,
                   hipStream_t s, const float *w32, float *rf, const XDefer &xq);
void launch_wdots(const Ctx &c, int64_t n, const double *w, int nd, const double *const *a,
                  const double *const *b, double *out, hipStream_t s, const float *w32 = nullptr);
// out[j] = (r, z_j)_w for FP32 z_0 (and z_1 when not null), on the device
void launch_wdots_rz(const Ctx &c, int64_t n, const double *w, const float *w32, const double *r,
                     const float *z0, const float *z1, double *out, hipStream_t s);
// p = z + beta p, beta = (rzn[0] (- rzn[1] when flexible)) / rzo[0] on the device
template <typename ZT>
void launch_zp(int64_t n, const ZT *z, const double *rzn, const double *rzo, bool flexible,
               double *p, hipStream_t s);
// block dots for Gram-Schmidt: out[j] = sum_i w_i V_j(i) x(i), j < k
void launch_mdot(const Ctx &c, int64_t n, const double *w, int k, const double *V, int64_t ld,
                 const double *x, double *out, hipStream_t s);
// x -= sum_j h_j V_j  (h on device)
void launch_mupdate(int64_t n, int k, const double *V, int64_t ld, const double *h, double *x,
                    double sign, hipStream_t s);
void launch_fill(int64_t n, double v, double *x, hipStream_t s);
template <typename T>
void launch_copy(int64_t n, const T *x, T *y, hipStream_t s);
void launch_fillf(int64_t n, float v, float *x, hipStream_t s);

// coarse PCG kernels with device scalars (blas.hip)
void launch_cpcg_init(const Ctx &c, const Level &L, double tol2, int maxit, hipStream_t s);
void launch_cpcg_iteration(const Ctx &c, const Level &L, bool first, hipStream_t s);

// transfer.hip
template <typename T>
void launch_prolong(const Level &F, const Level &C, const T *xc, T *xf, hipStream_t s, int nv = 1);
// bf != null: restrict bf - rf (the residual of a right side bf and a product rf)
template <typename T>
void launch_restrict(const Level &F, const Level &C, const T *rf, T *rc, hipStream_t s,
                     int nv = 1, const T *bf = nullptr);

// fdm.hip
void launch_fdm_setup(const Ctx &c, Level &L, hipStream_t s);
// rs (may be null): solve on r - rs (a residual formed as it is read)
// xin: 0 inputs assembled; 1 r, 2 rs comes without the x step of its
// gather-scatter (only where fdm_takes_x_step says the kernel can add it)
template <typename T>
void launch_fdm(const Ctx &c, const Level &L, const T *r, T *z, bool asm_mode, hipStream_t s,
                int nv = 1, const T *rs = nullptr, int xin = 0);
void launch_fdm_mfma(const Ctx &c, const Level &L, const float *r, float *z, bool asm_mode,
                     int prec, hipStream_t s, int nv = 1);
template <typename T>
void launch_asm_sum(const Ctx &c, const Level &L, const T *box, T *z, hipStream_t s);

// fdm_mf32.hip: FP32 RAS local solves on the matrix cores (2 <= p <= 9, no
// floating box)
bool fdm_mf32_supported(const Ctx &c, int p);
// prec: the operand format of the contractions (SEM_F32, or SEM_F16 /
// SEM_BF16 with the level's 16-bit factors)
void launch_fdm_mf32(const Ctx &c, const Level &L, const float *r, float *z, hipStream_t s, int nv,
                     const float *rs, int xin, int prec = SEM_F32);
// 32-bit words per element of L.A16 (degree p, 2 <= p <= 9), and its setup
// from L.S16
size_t mf16_table_words(int p);
void launch_fdm_mf16_pack(const Level &L, hipStream_t s);

// coarse.hip
// doubles of block partials the coarse Jacobi-PCG kernels need for n unknowns
size_t coarse_cg_partials(int64_t n);
bool coarse_assembled_ok(const Ctx &c, const Level &C);
void coarse_setup(Ctx &c, Level &C, hipStream_t s);
// The coarse right side as the restriction leaves it, before its
// gather-scatter (p null: C.d_b, assembled): the mapping to the global
// numbering then sums the copies of each node itself.
struct CoarseRhs {
  const void *p = nullptr;
  bool f32 = false;
};
void coarse_solve_assembled(Ctx &c, Level &C, double tol, int maxit, hipStream_t s, int nv = 1,
                            CoarseRhs u = {});
void coarse_release(CoarseSolver &S);
size_t coarse_direct_bytes(int64_t nx, int64_t ny, int64_t nz, bool f32);
void coarse_direct_setup(CoarseSolver &S, int64_t nx, int64_t ny, int64_t nz, hipStream_t s);
// nv right sides, S.n apart in b, x and the work vector S.dy
void coarse_direct_apply(const CoarseSolver &S, int64_t nx, int64_t ny, int64_t nz, const double *b,
                         double *x, hipStream_t s, int nv = 1);

// hessenberg.cpp
double hessenberg_max_abs_eig(const double *H, int ldh, int k);

}  // namespace sem
