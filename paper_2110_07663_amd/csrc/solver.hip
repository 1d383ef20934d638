// Setup, multigrid and Krylov drivers, and the C ABI of include/sem.h.
//
// Sec. 2.2 / 2.2.2 / 2.2.3 of arXiv:2110.07663: a single-pass p-multigrid
// V-cycle (Algorithm 1) with Chebyshev-accelerated (Algorithm 2) Jacobi or
// Schwarz smoothing, bounds (0.1, 1.1) lambda~ from Arnoldi on S A, inside
// flexible CG or flexible GMRES.  Every vector operation runs in the HIP
// kernels of this library; the host only sequences launches and reads back
// the few scalars the Krylov recurrences and the Arnoldi eigenvalue need.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "sem_internal.h"

namespace sem {

static thread_local std::string g_last_error;

void fail(sem_status st, const std::string &msg) { throw Error{st, msg}; }
void set_last_error(const std::string &msg) { g_last_error = msg; }

void check_hip(hipError_t e, const char *what, const char *file, int line) {
  if (e != hipSuccess) {
    char buf[512];
    snprintf(buf, sizeof(buf), "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    fail(SEM_EHIP, buf);
  }
}

template <typename F>
static sem_status guarded(F &&f) {
  try {
    f();
    return SEM_OK;
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return SEM_EHIP;
  } catch (...) {
    g_last_error = "unexpected exception";
    return SEM_EHIP;
  }
}

static inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// workspace layout (planning and setup walk the same sequence)
struct SetupScratch {
  double *xyz = nullptr, *xig = nullptr, *Jg = nullptr, *diag = nullptr;
  int *bad = nullptr;
  Arena gs;  // sort scratch, reset per level
};

static void validate(const sem_mesh *m, int p, const int8_t *bc, const sem_opts *o) {
  if (!m || !bc || !o) fail(SEM_EINVAL, "null mesh, bc or opts");
  if (m->nex < 1 || m->ney < 1 || m->nez < 1) fail(SEM_EINVAL, "element counts must be >= 1");
  if (m->p_geom < 1 || m->p_geom > kMaxP) fail(SEM_EINVAL, "p_geom must be in [1, 10]");
  if (p < 1) fail(SEM_EINVAL, "p must be >= 1");
  if (p > kMaxP) fail(SEM_EUNSUPPORTED, "p > 10 is not supported");
  if (o->precond == SEM_PRECOND_PMG) {
    if (o->nlevels < 1 || o->nlevels > kMaxLevels) fail(SEM_EINVAL, "nlevels must be in [1, 8]");
    if (o->p_levels[0] != p) fail(SEM_EINVAL, "p_levels[0] must equal p");
    for (int l = 1; l < o->nlevels; ++l)
      if (o->p_levels[l] >= o->p_levels[l - 1] || o->p_levels[l] < 1)
        fail(SEM_EINVAL, "p_levels must be strictly decreasing and >= 1");
    if (o->smoother != SEM_SMOOTH_JACOBI && o->smoother != SEM_SMOOTH_RAS &&
        o->smoother != SEM_SMOOTH_ASM)
      fail(SEM_EINVAL, "unknown smoother");
    if (o->smoother != SEM_SMOOTH_JACOBI)
      for (int l = 0; l + 1 < o->nlevels; ++l)
        if (o->p_levels[l] < 2) fail(SEM_EINVAL, "Schwarz smoothing needs p >= 2 on smoothed levels");
    if (o->cheb_order < 0 || o->cheb_order > 32) fail(SEM_EINVAL, "cheb_order out of range");
    if (!(o->lmax_fac > o->lmin_fac) || !(o->lmin_fac >= 0)) fail(SEM_EINVAL, "bad Chebyshev factors");
  } else if (o->precond != SEM_PRECOND_JACOBI) {
    fail(SEM_EINVAL, "unknown preconditioner");
  }
  if (o->smoother_prec != SEM_F64 && o->smoother_prec != SEM_F32)
    fail(SEM_EINVAL, "smoother_prec must be SEM_F64 or SEM_F32");
  if (o->fdm_prec < SEM_F64 || o->fdm_prec > SEM_F16) fail(SEM_EINVAL, "bad fdm_prec");
  if ((o->fdm_prec == SEM_BF16 || o->fdm_prec == SEM_F16) && o->smoother_prec != SEM_F32)
    fail(SEM_EINVAL, "BF16/FP16 FDM needs smoother_prec = SEM_F32");
  if (o->arnoldi_steps < 1 || o->arnoldi_steps > kMaxArnoldi) fail(SEM_EINVAL, "arnoldi_steps in [1,16]");
  if (o->krylov < SEM_KRYLOV_PCG || o->krylov > SEM_KRYLOV_FGMRES) fail(SEM_EINVAL, "bad krylov");
  if (o->krylov == SEM_KRYLOV_FGMRES && (o->gmres_restart < 1 || o->gmres_restart > kMaxRestart))
    fail(SEM_EINVAL, "gmres_restart in [1, 64]");
  if (o->coarse_maxit < 1) fail(SEM_EINVAL, "coarse_maxit must be >= 1");
  if (o->ax_variant < -1 || o->ax_variant > 2) fail(SEM_EINVAL, "ax_variant must be in [-1, 2]");
  if (o->batch_rhs < 0 || o->batch_rhs > 64) fail(SEM_EINVAL, "batch_rhs must be in [0, 64]");
  if (o->coarse_solver < -1 || o->coarse_solver > 1) fail(SEM_EINVAL, "coarse_solver must be in [-1, 1]");
  if (o->proj_max < 0 || o->proj_max > 32) fail(SEM_EINVAL, "proj_max must be in [0, 32]");
  if (o->geom_prec != SEM_F32 && o->geom_prec != SEM_F16)
    fail(SEM_EINVAL, "geom_prec must be SEM_F32 or SEM_F16");
  if (o->geom_prec == SEM_F16 && o->smoother_prec != SEM_F32)
    fail(SEM_EINVAL, "FP16 geometric factors need smoother_prec = SEM_F32");
  for (int f = 0; f < 6; ++f)
    if (bc[f] != 0 && bc[f] != 1) fail(SEM_EINVAL, "bc flags must be 0 or 1");
  int64_t E = (int64_t)m->nex * m->ney * m->nez;
  int64_t nloc = E * (p + 1) * (p + 1) * (p + 1);
  if (nloc >= (int64_t)1 << 31) fail(SEM_EUNSUPPORTED, "more than 2^31 local nodes");
}

// carve every buffer; with a null arena base this only sizes the workspace
static void layout(Ctx &c, const sem_mesh *m, Arena &A, SetupScratch &sc) {
  const sem_opts &o = c.opts;
  const bool lowp = c.lowp;
  const bool schwarz = o.precond == SEM_PRECOND_PMG && o.smoother != SEM_SMOOTH_JACOBI;
  const bool asm_on = schwarz && o.smoother == SEM_SMOOTH_ASM;
  // batch lanes share one V-cycle when the hierarchy ends in the assembled
  // p = 1 solve: every level's work vectors then hold all lanes
  c.nlanes = std::max(0, o.batch_rhs);
  c.nvmax = (c.nlanes > 1 && o.precond == SEM_PRECOND_PMG && c.nlev > 1 &&
             c.lev[c.nlev - 1].p == 1)
                ? c.nlanes
                : 1;
  const size_t nv = (size_t)c.nvmax;
  for (int l = 0; l < c.nlev; ++l) {
    Level &L = c.lev[l];
    const bool smoothed = !L.coarse;
    L.xi = A.take<double>(L.N);
    L.wq = A.take<double>(L.N);
    L.D64 = A.take<double>(L.N * L.N);
    L.D32 = A.take<float>(L.N * L.N);
    if (l + 1 < c.nlev) {
      L.J64 = A.take<double>(L.N * c.lev[l + 1].N);
      L.J32 = A.take<float>(L.N * c.lev[l + 1].N);
    }
    L.X = A.take<double>(3 * L.nloc);
    L.G64 = A.take<double>(6 * L.nloc);
    if (lowp) L.G32 = A.take<float>(6 * L.nloc);
    if (lowp && o.geom_prec == SEM_F16 && smoothed) {
      L.G16 = A.take<uint32_t>(3 * L.nloc);
      L.gscale = A.take<float>(L.E);
    }
    if (L.fine) L.BL = A.take<double>(L.nloc);
    if (L.fine) L.dotpart = A.take<double>(L.E);
    L.w64 = A.take<double>(L.nloc);
    if (lowp) L.w32 = A.take<float>(L.nloc);
    L.dinv64 = A.take<double>(L.nloc);
    if (lowp) L.dinv32 = A.take<float>(L.nloc);
    L.perm = A.take<int32_t>(L.nloc);
    L.off = A.take<int32_t>(L.nglob + 1);
    if (schwarz && smoothed) {
      int pb = L.pb;
      L.boxlen = A.take<double>(3 * L.E);
      L.S64 = A.take<double>(3 * L.E * pb * pb);
      L.lam64 = A.take<double>(3 * L.E * pb);
      if (lowp) {
        L.S32 = A.take<float>(3 * L.E * pb * pb);
        L.lam32 = A.take<float>(3 * L.E * pb);
        if (o.fdm_prec == SEM_BF16 || o.fdm_prec == SEM_F16) {
          L.S16 = A.take<uint16_t>(3 * L.E * pb * pb);
          L.sscale = A.take<float>(3 * L.E);
          if (L.p >= 2 && L.p <= 9) L.A16 = A.take<uint32_t>(L.E * mf16_table_words(L.p));
        }
      }
      if (asm_on) {
        L.box64 = A.take<double>(L.E * pb * pb * pb);
        if (lowp) L.box32 = A.take<float>(L.E * pb * pb * pb);
      }
    }
    // FP64 work vectors: every right side where the V-cycle runs in FP64 (and
    // on the coarsest level, whose solve is FP64), else one
    const size_t nd = (!lowp || L.coarse) ? nv : 1;
    L.d_b = A.take<double>(nd * L.nloc);
    L.d_x = A.take<double>(nd * L.nloc);
    L.d_r = A.take<double>(nd * L.nloc);
    L.d_d = A.take<double>(nd * L.nloc);
    L.d_w = A.take<double>(nd * L.nloc);
    L.d_t = A.take<double>(nd * L.nloc);
    if (lowp) {
      L.f_b = A.take<float>(nv * L.nloc);
      L.f_x = A.take<float>(nv * L.nloc);
      L.f_r = A.take<float>(nv * L.nloc);
      L.f_d = A.take<float>(nv * L.nloc);
      L.f_w = A.take<float>(nv * L.nloc);
      L.f_t = A.take<float>(nv * L.nloc);
    }
  }
  c.partials = A.take<double>(kRedBlocks * 8);
  c.counter = A.take<unsigned>(64);
  c.dres = A.take<double>(2 * kMaxRestart + 64);
  c.dsc = A.take<DevScalars>(1);
  const Level &F = c.lev[0];
  c.kr = A.take<double>(F.nloc);
  c.kz = A.take<double>(F.nloc);
  c.kzold = A.take<double>(F.nloc);
  c.kp = A.take<double>(F.nloc);
  c.kq = A.take<double>(F.nloc);
  c.kx = A.take<double>(F.nloc);
  c.fzo = nullptr;
  if (lowp && o.precond == SEM_PRECOND_PMG && c.nlev > 1) c.fzo = A.take<float>(nv * F.nloc);
  if (o.krylov == SEM_KRYLOV_FGMRES) {
    c.gV = A.take<double>((size_t)(o.gmres_restart + 1) * F.nloc);
    c.gZ = A.take<double>((size_t)o.gmres_restart * F.nloc);
  }
  c.nproj = 0;
  if (o.proj_max > 0) {
    c.projX = A.take<double>((size_t)o.proj_max * F.nloc);
    c.projAX = A.take<double>((size_t)o.proj_max * F.nloc);
    c.projW = A.take<double>(F.nloc);
    c.projAW = A.take<double>(F.nloc);
  }
  const Level &C = c.lev[c.nlev - 1];
  c.cx = A.take<double>(nv * C.nloc);
  c.cr = A.take<double>(C.nloc);
  c.cz = A.take<double>(C.nloc);
  c.cp = A.take<double>(C.nloc);
  c.cq = A.take<double>(C.nloc);
  if (o.precond == SEM_PRECOND_PMG && c.nlev > 1)
    c.av = A.take<double>((size_t)(o.arnoldi_steps + 1) * F.nloc);
  // batched-solve lanes
  if (c.nlanes > 0) {
    c.lanev = A.take<double>((size_t)c.nlanes * 5 * F.nloc);
    c.lanes = A.take<char>((size_t)c.nlanes * 128);
    c.lpartials = A.take<double>((size_t)c.nlanes * kRedBlocks * 8);
  }
  // assembled coarse solve when the coarsest level is p = 1
  c.cs = nullptr;
  if (o.precond == SEM_PRECOND_PMG && C.p == 1) {
    CoarseSolver &S = c.coarse_store;
    S.n = C.nglob;
    S.St = A.take<double>(27 * S.n);
    S.dinv = A.take<double>(S.n);
    S.Ae = A.take<double>(64 * C.E);
    S.b = A.take<double>(nv * S.n);
    S.x = A.take<double>(nv * S.n);
    S.r = A.take<double>(S.n);
    S.u = A.take<double>(S.n);
    S.w = A.take<double>(S.n);
    S.p = A.take<double>(S.n);
    S.s = A.take<double>(S.n);
    S.r2 = A.take<double>(S.n);
    S.w2 = A.take<double>(S.n);
    S.s2 = A.take<double>(S.n);
    S.partials = A.take<double>(coarse_cg_partials(S.n));
    // exact block-tridiagonal solve of the p = 1 level (chosen, or by size)
    {
      const int64_t nx = m->nex + 1, ny = m->ney + 1, nz = m->nez + 1;
      // FP32 smoother: the sweeps read FP32 copies of the blocks (SEM_COARSE_F64=1 keeps FP64)
      const char *cf = getenv("SEM_COARSE_F64");
      const bool f32 = lowp && !(cf && cf[0] == '1');
      const size_t db = coarse_direct_bytes(nx, ny, nz, false);
      const bool want = o.coarse_solver == 1 || (o.coarse_solver < 0 && db <= ((size_t)4 << 30));
      S.direct = false;
      S.dG = S.dH = S.dJ = S.dy = nullptr;
      S.fG = S.fH = S.fJ = nullptr;
      S.dflag = nullptr;
      if (want) {
        const int64_t Mp = (nx * ny + 31) / 32 * 32;
        S.dG = A.take<double>((size_t)(nz * Mp * Mp));
        S.dH = A.take<double>((size_t)(nz * Mp * Mp));
        S.dJ = A.take<double>((size_t)(nz * Mp * Mp));
        if (f32) {
          S.fG = A.take<float>((size_t)(nz * Mp * Mp));
          S.fH = A.take<float>((size_t)(nz * Mp * Mp));
          S.fJ = A.take<float>((size_t)(nz * Mp * Mp));
        }
        S.dy = A.take<double>(std::max<size_t>(nv * S.n, Mp));  // also the pivot-test diagonal
        S.dflag = A.take<int>(64);
        S.direct = true;  // until the setup finds the level singular
      }
    }
    S.counter = A.take<unsigned>(64);
    S.sc = A.take<CoarseScalars>(1);
    const char *g = getenv("SEM_COARSE_GRAPH");
    S.use_graph = !(g && g[0] == '0');
    c.cs = &S;
  }
  // setup-only scratch
  int Ng = m->p_geom + 1;
  int64_t E = F.E;
  sc.xyz = A.take<double>((size_t)E * Ng * Ng * Ng * 3);
  sc.xig = A.take<double>(Ng);
  sc.Jg = A.take<double>(Ng * (kMaxP + 1));
  sc.bad = A.take<int>(64);
  size_t gsb = 8 * (F.nloc + 1) * sizeof(int32_t) + 16 + gs_sort_temp_bytes(F.nloc) + 12 * 256;
  char *g = A.take<char>(gsb);
  sc.gs.base = g;
  sc.gs.cap = gsb;
}

static void init_ctx(Ctx &c, const sem_mesh *m, int p, const int8_t *bc, const sem_opts *o) {
  c.nex = m->nex;
  c.ney = m->ney;
  c.nez = m->nez;
  for (int f = 0; f < 6; ++f) c.bc[f] = bc[f];
  c.opts = *o;
  c.lowp = o->smoother_prec == SEM_F32;
  c.fdm_prec = o->fdm_prec == SEM_F64 ? (c.lowp ? SEM_F32 : SEM_F64) : o->fdm_prec;
  if (c.fdm_prec == SEM_F64 && c.lowp) c.fdm_prec = SEM_F32;
  if (o->precond == SEM_PRECOND_JACOBI) {
    c.nlev = 1;
    c.opts.p_levels[0] = p;
  } else {
    c.nlev = o->nlevels;
  }
  int64_t E = (int64_t)m->nex * m->ney * m->nez;
  for (int l = 0; l < c.nlev; ++l) {
    Level &L = c.lev[l];
    L = Level();
    L.p = c.opts.p_levels[l];
    L.N = L.p + 1;
    L.N3 = L.N * L.N * L.N;
    L.pb = L.p + 3;
    L.E = E;
    L.nloc = E * L.N3;
    L.nglob = ((int64_t)m->nex * L.p + 1) * ((int64_t)m->ney * L.p + 1) * ((int64_t)m->nez * L.p + 1);
    L.fine = l == 0;
    L.coarse = l == c.nlev - 1;
    L.nex = m->nex;
    L.ney = m->ney;
    L.nez = m->nez;
    for (int f = 0; f < 6; ++f) L.bc[f] = bc[f];
    {  // SEM_GS_SORTED=1: the sorted-segment gather-scatter instead of the direction passes
      const char *gsv = getenv("SEM_GS_SORTED");
      L.gs_struct = !(gsv && gsv[0] == '1');
      // SEM_AX_XFUSE=0: the p = 7 Ax leaves every x-face to the gather-scatter
      const char *xfv = getenv("SEM_AX_XFUSE");
      L.xfuse = !(xfv && xfv[0] == '0');
      // SEM_GS_XDEFER=0: the gather-scatter after an FDM that only feeds a
      // Chebyshev update takes its x step itself
      const char *xdv = getenv("SEM_GS_XDEFER");
      L.xdefer = !(xdv && xdv[0] == '0');
      // SEM_GS_YDEFER=0: ... its x step only (y and z passes run)
      const char *ydv = getenv("SEM_GS_YDEFER");
      L.ydefer = !(ydv && ydv[0] == '0');
      // SEM_GS_YZ=0 / 1: the y and z passes as two launches / one launch in
      // both precisions (default: one launch for FP64, measured faster there
      // and slower in FP32)
      const char *yzv = getenv("SEM_GS_YZ");
      L.gs_yz = yzv ? (yzv[0] == '1' ? 1 : 0) : -1;
    }
    L.lowp = c.lowp;
    // Ax kernel shape at p = 7 (option, else SEM_AX_VARIANT, else one wave/element,
    // non-temporal streams)
    const char *av = getenv("SEM_AX_VARIANT");
    L.ax_variant = o->ax_variant >= 0 ? o->ax_variant : (av ? atoi(av) : 2);
  }
  const char *fl = getenv("SEM_FDM_LINES");
  c.fdm_lines = !(fl && fl[0] == '0');
  const char *fg = getenv("SEM_FDM_GROUP");
  c.fdm_group = !(fg && fg[0] == '0');
  const char *fm = getenv("SEM_FDM_MFMA1");
  c.fdm_mfma1 = fm && fm[0] == '1';
  const char *f32 = getenv("SEM_FDM_MF32");
  c.fdm_mf32 = !(f32 && f32[0] == '0');
  const char *f16 = getenv("SEM_FDM_MF16");
  c.fdm_mf16 = !(f16 && f16[0] == '0');
  const char *fch = getenv("SEM_FDM_MF32_CHAIN");
  c.fdm_mf32_chain = fch && fch[0] == '2' ? 2 : 1;
  const char *fxs = getenv("SEM_FDM_XSTEP");
  c.fdm_xstep = !(fxs && fxs[0] == '0');
  const char *fys = getenv("SEM_FDM_YSTEP");
  c.fdm_ystep = !(fys && fys[0] == '0');
  const char *fxf = getenv("SEM_FDM_XFACES");
  c.fdm_xfaces = !(fxf && fxf[0] == '0');
  const char *csm = getenv("SEM_COARSE_SUM");
  c.coarse_sum = !(csm && csm[0] == '0');
}

// ---------------------------------------------------------------------------
// operator pieces in precision T
template <typename T>
struct Vec;
template <>
struct Vec<double> {
  static double *b(Level &L) { return L.d_b; }
  static double *x(Level &L) { return L.d_x; }
  static double *r(Level &L) { return L.d_r; }
  static double *d(Level &L) { return L.d_d; }
  static double *w(Level &L) { return L.d_w; }
  static double *t(Level &L) { return L.d_t; }
  static const double *dinv(const Level &L) { return L.dinv64; }
};
template <>
struct Vec<float> {
  static float *b(Level &L) { return L.f_b; }
  static float *x(Level &L) { return L.f_x; }
  static float *r(Level &L) { return L.f_r; }
  static float *d(Level &L) { return L.f_d; }
  static float *w(Level &L) { return L.f_w; }
  static float *t(Level &L) { return L.f_t; }
  static const float *dinv(const Level &L) { return L.dinv32; }
};

size_t Profiler::begin(int kind, hipStream_t s) {
  if (used == pool.size()) {
    // timing only: no system-scope fence (cache write-back and invalidation)
    // when an event is recorded, so the instrumented solve runs as it would
    hipEvent_t a, b;
    SEM_HIP(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
    SEM_HIP(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
    pool.push_back({a, b});
  }
  Rec r{kind, pool[used].first, pool[used].second};
  ++used;
  SEM_HIP(hipEventRecord(r.a, s));
  recs.push_back(r);
  return recs.size() - 1;
}
void Profiler::end(size_t rec, hipStream_t s) { (void)hipEventRecord(recs[rec].b, s); }
void Profiler::reset() {
  recs.clear();
  used = 0;
}
Profiler::~Profiler() {
  for (auto &e : pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
}

// records the enclosed launches when profiling a finest-level kernel
// (scopes nest: each closes its own record)
struct ProfScope {
  Profiler *p;
  hipStream_t s;
  size_t rec = 0;
  ProfScope(const Ctx &c, const Level &L, int kind, hipStream_t st)
      : p((c.prof && c.prof->on && ((c.prof->kinds >> kind) & 1u) && !c.capturing &&
           (L.fine || kind >= SEM_PROF_COARSE))
              ? c.prof
              : nullptr),
        s(st) {
    if (p) rec = p->begin(kind, s);
  }
  ~ProfScope() {
    if (p) p->end(rec, s);
  }
};

// nv right sides, nloc apart (batch lanes sharing a V-cycle); 1 otherwise
template <typename T>
static void opA(const Ctx &c, const Level &L, const T *u, T *Au, hipStream_t s, int nv = 1,
                double *dotp = nullptr) {
  const bool xf = ax_sums_x_faces(L);  // Ax sums the x-faces inside its workgroups
  {
    ProfScope ps(c, L, sizeof(T) == 8 ? SEM_PROF_AX64 : SEM_PROF_AX32, s);
    launch_ax<T>(L, u, Au, s, nv, xf, dotp);
  }
  ProfScope ps(c, L, sizeof(T) == 8 ? SEM_PROF_GS64 : SEM_PROF_GS32, s);
  launch_gs<T>(L, Au, s, nv, xf);
}

// q = A p and (p, q) into *pq (device).  For p consistent and zero on the
// Dirichlet nodes (every search direction of the CG drivers) the p = 7 FP64 Ax
// forms (p, q) from its element shares of p^T A_L p; else a weighted dot.
//
// q only feeds the FCG update (the dot comes from the element shares), so
// when the vectors allow, its gather-scatter runs the z pass only and the
// update takes the x and y steps as it reads q (*xq says so).
static void opA_dot(const Ctx &c, const Level &L, const double *p, double *q, double *pq,
                    hipStream_t s, XDefer *xq = nullptr) {
  if (L.dotpart && ax_forms_dot(L, 1)) {
    if (xq && L.gs_struct && L.xdefer && L.ydefer && L.w32 &&
        cheb_can_defer_x<double>(L.N, L.nloc, {p, q, L.w32})) {
      {
        ProfScope ps(c, L, SEM_PROF_AX64, s);
        launch_ax<double>(L, p, q, s, 1, false, L.dotpart);
      }
      {
        ProfScope ps(c, L, SEM_PROF_GS64, s);
        launch_gs<double>(L, q, s, 1, false, true, true);
      }
      xq->on = true;
      xq->nex = L.nex;
      xq->N = L.N;
      xq->bc0 = L.bc[0];
      xq->bc1 = L.bc[1];
      xq->nloc = L.nloc;
      xq->y = true;
      xq->ney = L.ney;
      xq->bc2 = L.bc[2];
      xq->bc3 = L.bc[3];
    } else {
      opA<double>(c, L, p, q, s, 1, L.dotpart);
    }
    launch_sum_partials(L.E, L.dotpart, pq, s);
    return;
  }
  opA<double>(c, L, p, q, s);
  const double *a[1] = {p}, *bb[1] = {q};
  launch_wdots(c, L.nloc, L.w64, 1, a, bb, pq, s, L.w32);
}

// rs (may be null): apply S to r - rs; r - rs is formed as the VALU FDM reads
// it, else stored into rs first
// xd (may be null): when the result only feeds a Chebyshev update, the x step
// of the gather-scatter may be left to that update (xd->on says so)
// Whether the level's Schwarz smoother in precision T reads A's output with
// the x step of its gather-scatter left out and takes that step itself (the
// FP32 matrix-core RAS kernel); then the products that only feed it skip it.
// Whether the level's RAS local solves run in the matrix-core line kernel
// (fdm_mf32.hip): FP32 operands, or FP16 / BF16 operands in its 4x4x4 form
// (otherwise the 16-bit tile kernel of fdm_mfma.hip)
static bool fdm_in_mf(const Ctx &c, const Level &L) {
  const bool b16 = c.fdm_prec == SEM_BF16 || c.fdm_prec == SEM_F16;
  return (b16 ? c.fdm_mf16 && L.A16 && L.sscale : c.fdm_mf32) &&
         c.opts.smoother == SEM_SMOOTH_RAS && !L.coarse && fdm_mf32_supported(c, L.p);
}

template <typename T>
static bool fdm_takes_x_step(const Ctx &c, const Level &L) {
  return sizeof(T) == 4 && c.fdm_xstep && c.opts.precond == SEM_PRECOND_PMG && fdm_in_mf(c, L) &&
         L.gs_struct;
}

// ... and the y step too: only the z step of A's gather-scatter is taken
template <typename T>
static bool fdm_takes_y_step(const Ctx &c, const Level &L) {
  return fdm_takes_x_step<T>(c, L) && c.fdm_ystep;
}

// Whether the FP32 matrix-core RAS kernel sums the x-faces its workgroup
// shares (four consecutive elements along x) before it stores
template <typename T>
static bool fdm_sums_x_faces(const Ctx &c, const Level &L) {
  return sizeof(T) == 4 && c.fdm_xfaces && fdm_in_mf(c, L) && L.gs_struct && L.nex % 4 == 0 &&
         L.E % 4 == 0;
}

// A u with the x step (and, when the smoother takes it, the y step) of the
// gather-scatter left to the reader
template <typename T>
static void opA_nox(const Ctx &c, const Level &L, const T *u, T *Au, hipStream_t s, int nv) {
  {
    ProfScope ps(c, L, sizeof(T) == 8 ? SEM_PROF_AX64 : SEM_PROF_AX32, s);
    launch_ax<T>(L, u, Au, s, nv, false, nullptr);
  }
  ProfScope ps(c, L, sizeof(T) == 8 ? SEM_PROF_GS64 : SEM_PROF_GS32, s);
  launch_gs<T>(L, Au, s, nv, false, true, fdm_takes_y_step<T>(c, L));
}

// xin: 0 r and rs assembled; 1 r, 2 rs comes from opA_nox (fdm_takes_x_step),
// + 4 when opA_nox left the y step as well (fdm_takes_y_step)
template <typename T>
static void opS(const Ctx &c, const Level &L, const T *r, T *z, hipStream_t s, int nv = 1,
                T *rs = nullptr, XDefer *xd = nullptr, int xin = 0) {
  const bool schwarz = c.opts.precond == SEM_PRECOND_PMG && c.opts.smoother != SEM_SMOOTH_JACOBI &&
                       !L.coarse;
  const bool asm_mode = c.opts.smoother == SEM_SMOOTH_ASM;
  const bool b16 = sizeof(T) == 4 && (c.fdm_prec == SEM_BF16 || c.fdm_prec == SEM_F16);
  const bool mf16 = b16 && !asm_mode && fdm_in_mf(c, L);  // 16-bit line kernel
  const bool mfma = b16 && !mf16;                         // 16-bit tile kernel
  if (xin && !fdm_takes_x_step<T>(c, L)) fail(SEM_EINVAL, "smoother: inputs must be assembled");
  if (rs && (!schwarz || asm_mode || mfma)) {  // form r - rs in rs, then apply S to it
    launch_sub<T>(L.nloc * nv, r, rs, rs, s);
    r = rs;
    rs = nullptr;
  }
  if (!schwarz) {
    const T *dinv = Vec<T>::dinv(L);
    if (!dinv) fail(SEM_EINVAL, "Jacobi data of this precision were not built");
    for (int k = 0; k < nv; ++k) launch_scale<T>(L.nloc, dinv, r + k * L.nloc, z + k * L.nloc, s);
    return;
  }
  // S's output may leave the x step of its gather-scatter to a reader (xd),
  // or arrive with the x-faces inside each FDM workgroup summed
  const bool defer = !asm_mode && xd && L.gs_struct && L.xdefer &&
                     cheb_can_defer_x<T>(L.N, L.nloc * nv, {z});
  const bool fxf = !asm_mode && !defer && !mfma && (xin & 3) != 1 && fdm_sums_x_faces<T>(c, L);
  {
    ProfScope ps(c, L, SEM_PROF_FDM, s);
    if constexpr (sizeof(T) == 4) {
      if (mfma) launch_fdm_mfma(c, L, (const float *)r, (float *)z, asm_mode, c.fdm_prec, s, nv);
      if (mf16)
        launch_fdm_mf32(c, L, (const float *)r, (float *)z, s, nv, (const float *)rs,
                        xin | (fxf ? 8 : 0), c.fdm_prec);
    }
    if (!mfma && !mf16) launch_fdm<T>(c, L, r, z, asm_mode, s, nv, rs, xin | (fxf ? 8 : 0));
  }
  if (asm_mode) return;  // the overlap sum already produced a consistent, masked vector
  if (defer) {
    xd->on = true;
    xd->nex = L.nex;
    xd->N = L.N;
    xd->bc0 = L.bc[0];
    xd->bc1 = L.bc[1];
    xd->nloc = L.nloc;
    xd->y = L.ydefer;
    xd->ney = L.ney;
    xd->bc2 = L.bc[2];
    xd->bc3 = L.bc[3];
  }
  ProfScope ps(c, L, sizeof(T) == 8 ? SEM_PROF_GS64 : SEM_PROF_GS32, s);
  launch_gs<T>(L, z, s, nv, fxf, defer, defer && L.ydefer);
}

// Algorithm 2 read as a correction: x <- x + e (x_zero: x <- e)
template <typename T>
static void chebyshev(const Ctx &c, Level &L, const T *b, T *x, bool x_zero, hipStream_t s,
                      int nv = 1) {
  T *r = Vec<T>::r(L), *d = Vec<T>::d(L), *w = Vec<T>::w(L), *t = Vec<T>::t(L);
  const double theta = 0.5 * (L.lmax + L.lmin), delta = 0.5 * (L.lmax - L.lmin);
  const double sigma = theta / delta;
  const int64_t n = L.nloc * nv;  // the vector updates are pointwise over all right sides
  double rho = 1.0 / sigma;
  // A's output that only feeds S may leave the x step of its gather-scatter to S
  const bool xs = fdm_takes_x_step<T>(c, L);
  const int ys = fdm_takes_y_step<T>(c, L) ? 4 : 0;
  if (x_zero) {
    opS<T>(c, L, b, r, s, nv);
  } else if (xs) {
    opA_nox<T>(c, L, x, w, s, nv);
    opS<T>(c, L, b, r, s, nv, w, nullptr, 2 | ys);  // r = S (b - A x)
  } else {
    opA<T>(c, L, x, w, s, nv);
    opS<T>(c, L, b, r, s, nv, w);  // r = S (b - A x)
  }
  if (L.K == 0) {  // no acceleration: the smoother alone, x += S (b - A x)
    if (x_zero)
      launch_copy<T>(n, r, x, s);
    else
      launch_axpby<T>(n, (T)1, r, (T)1, x, s);
    return;
  }
  // pass 0 works from r_0 itself (d_0 = r_0 / theta is formed inside the update,
  // A and S being linear); a zero start is not written
  for (int k = 0; k < L.K; ++k) {
    if (xs)
      opA_nox<T>(c, L, k == 0 ? r : d, w, s, nv);
    else
      opA<T>(c, L, k == 0 ? r : d, w, s, nv);
    XDefer xd;  // t only feeds the update below: it may take the x step itself
    opS<T>(c, L, w, t, s, nv, nullptr, cheb_can_defer_x<T>(L.N, n, {x, r, d, t}) ? &xd : nullptr,
           xs ? 1 | ys : 0);
    double rho_new = 1.0 / (2.0 * sigma - rho);
    const T a = (T)(rho_new * rho), cc = (T)(2.0 * rho_new / delta);
    const bool last = k + 1 == L.K;
    if (k == 0)
      launch_cheb_first<T>(n, x, r, d, t, (T)(1.0 / theta), a, cc, x_zero, last, s, xd);
    else if (!last)
      launch_cheb_update<T>(n, x, r, d, t, a, cc, s, false, xd);
    else  // last pass and the closing x += d together
      launch_cheb_last<T>(n, x, r, d, t, a, cc, s, false, xd);
    rho = rho_new;
  }
}

static void host_scalars(Ctx &c, const void *dev, size_t bytes, hipStream_t s) {
  SEM_HIP(hipMemcpyAsync(c.hres, dev, bytes, hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
}

// coarse Jacobi-PCG from x = 0: C.d_b -> c.cx (all scalars on the device);
// u.p: the right side as the restriction left it (assembled solver only)
static void coarse_solve(Ctx &c, Level &C, hipStream_t s, int nv = 1, CoarseRhs u = {}) {
  const double tol = c.opts.coarse_tol;
  const int maxit = c.opts.coarse_maxit;
  ProfScope ps(c, C, SEM_PROF_COARSE, s);
  if (coarse_assembled_ok(c, C)) {
    coarse_solve_assembled(c, C, tol, maxit, s, nv, u);
    return;
  }
  if (u.p) fail(SEM_EINVAL, "coarse solve: the right side must be assembled");
  if (nv != 1) fail(SEM_EUNSUPPORTED, "several right sides need the assembled p = 1 coarse solve");
  DevScalars init{};
  init.tol2 = tol * tol;
  init.maxit = maxit;
  launch_cpcg_init(c, C, init.tol2, maxit, s);
  int done_iters = 0;
  bool first = true;
  if (tol <= 0.0 || c.capturing) {
    const int n = c.capturing && tol > 0.0 ? std::min(maxit, c.capture_coarse_iters) : maxit;
    for (int it = 0; it < n; ++it) {
      launch_cpcg_iteration(c, C, first, s);
      first = false;
    }
    if (!c.capturing) c.last_coarse_iters = maxit;
    return;
  }
  int chunk = std::max(8, c.last_coarse_iters + 2);
  while (true) {
    int n = std::min(chunk, maxit - done_iters);
    for (int it = 0; it < n; ++it) {
      launch_cpcg_iteration(c, C, first, s);
      first = false;
    }
    done_iters += n;
    host_scalars(c, c.dsc, sizeof(DevScalars), s);
    const DevScalars *h = reinterpret_cast<const DevScalars *>(c.hres);
    if (h->done || done_iters >= maxit) {
      c.last_coarse_iters = h->iters;
      if (!(h->rr == h->rr)) fail(SEM_ENAN, "NaN in the coarse-grid solve");
      return;
    }
    chunk = 8;
  }
}

// Whether level C's right side may reach the coarse solve as the restriction
// leaves it: the assembled solver's mapping to its global numbering then sums
// the copies of each node (no gather-scatter, no FP64 copy on the level)
static bool coarse_sums_restricted(const Ctx &c, const Level &C) {
  return c.coarse_sum && C.coarse && coarse_assembled_ok(c, C);
}

// one V-cycle of Algorithm 1 from x = 0 on level l (levels l.. in precision T);
// unassembled: the coarse level's right side is not yet assembled
template <typename T>
static void vcycle_level(Ctx &c, int l, hipStream_t s, int nv = 1, bool unassembled = false) {
  Level &L = c.lev[l];
  const int64_t n = L.nloc * nv;
  if (L.coarse) {
    if (unassembled) {
      coarse_solve(c, L, s, nv, CoarseRhs{Vec<T>::b(L), sizeof(T) == 4});
    } else {
      if constexpr (sizeof(T) == 4) launch_copy_cvt_f2d(n, L.f_b, L.d_b, s);
      coarse_solve(c, L, s, nv);
    }
    if constexpr (sizeof(T) == 4)
      launch_copy_cvt_d2f(n, c.cx, L.f_x, s);
    else
      launch_copy<double>(n, c.cx, L.d_x, s);
    return;
  }
  Level &C = c.lev[l + 1];
  T *b = Vec<T>::b(L), *x = Vec<T>::x(L), *w = Vec<T>::w(L);
  const bool csum = coarse_sums_restricted(c, C);
  if (L.K == 0) {  // smoother without acceleration: additive cycle, x = S b + P V(P^T b)
    opS<T>(c, L, b, x, s, nv);
    launch_restrict<T>(L, C, b, Vec<T>::b(C), s, nv);
    if (!csum) launch_gs<T>(C, Vec<T>::b(C), s, nv);
    vcycle_level<T>(c, l + 1, s, nv, csum);
    launch_prolong<T>(L, C, Vec<T>::x(C), x, s, nv);
    return;
  }
  chebyshev<T>(c, L, b, x, true, s, nv);                // x = M b
  opA<T>(c, L, x, w, s, nv);                            // r_C = P^T (b - A x)
  launch_restrict<T>(L, C, w, Vec<T>::b(C), s, nv, b);
  if (!csum) launch_gs<T>(C, Vec<T>::b(C), s, nv);
  vcycle_level<T>(c, l + 1, s, nv, csum);               // e_C
  launch_prolong<T>(L, C, Vec<T>::x(C), x, s, nv);      // x += P e_C
  chebyshev<T>(c, L, b, x, false, s, nv);               // post-smoothing
}

// z = M r on the finest level, FP64 in and out; nv right sides nloc apart
static void precondition(Ctx &c, const double *r, double *z, hipStream_t s, int nv = 1) {
  Level &F = c.lev[0];
  ProfScope ps(c, F, SEM_PROF_VCYCLE, s);
  if (nv < 1 || nv > c.nvmax) fail(SEM_EINVAL, "preconditioner: more right sides than were set up");
  const int64_t n = F.nloc * nv;
  if (c.opts.precond == SEM_PRECOND_JACOBI) {
    for (int k = 0; k < nv; ++k)
      launch_scale<double>(F.nloc, F.dinv64, r + k * F.nloc, z + k * F.nloc, s);
    return;
  }
  if (F.coarse) {  // single-level schedule: the coarse solve itself, on FP64 vectors
    launch_copy<double>(n, r, F.d_b, s);
    coarse_solve(c, F, s, nv);
    launch_copy<double>(n, c.cx, z, s);
    return;
  }
  if (c.lowp) {
    launch_copy_cvt_d2f(n, r, F.f_b, s);
    vcycle_level<float>(c, 0, s, nv);
    launch_copy_cvt_f2d(n, F.f_x, z, s);
  } else {
    launch_copy<double>(n, r, F.d_b, s);
    vcycle_level<double>(c, 0, s, nv);
    launch_copy<double>(n, F.d_x, z, s);
  }
}

// Mixed path: z = M r is the exact FP64 widening of the V-cycle's FP32 output,
// so the outer iteration keeps it in FP32 (F.f_x, and the previous one in
// c.fzo, swapped each iteration) instead of storing an FP64 copy.
static bool z_in_f32(const Ctx &c) {
  return c.lowp && c.fzo && c.opts.precond == SEM_PRECOND_PMG && !c.lev[0].coarse;
}
static void precondition_f32(Ctx &c, const double *r, hipStream_t s, bool have_f32 = false) {
  Level &F = c.lev[0];
  ProfScope ps(c, F, SEM_PROF_VCYCLE, s);
  if (!have_f32) launch_copy_cvt_d2f(F.nloc, r, F.f_b, s);  // else F.f_b holds it already
  vcycle_level<float>(c, 0, s);
}

// weighted dots on the finest level, read back to the host
static void dots(Ctx &c, const Level &L, int nd, const double *const *a, const double *const *b,
                 double *out, hipStream_t s) {
  launch_wdots(c, L.nloc, L.w64, nd, a, b, c.dres, s, L.w32);
  host_scalars(c, c.dres, nd * sizeof(double), s);
  for (int j = 0; j < nd; ++j) {
    out[j] = c.hres[j];
    if (!std::isfinite(out[j])) fail(SEM_ENAN, "NaN/Inf in an inner product");
  }
}

static double wnorm(Ctx &c, const Level &L, const double *v, hipStream_t s) {
  const double *a[1] = {v};
  double r;
  dots(c, L, 1, a, a, &r, s);
  return std::sqrt(r);
}

// ---------------------------------------------------------------------------
// Arnoldi on S A (FP64), lambda~ = largest |Ritz value|
static double arnoldi(Ctx &c, int l, hipStream_t s) {
  Level &L = c.lev[l];
  const int m = c.opts.arnoldi_steps;
  const int64_t ld = c.lev[0].nloc;
  double *V = c.av;
  std::vector<double> H((kMaxArnoldi + 1) * kMaxArnoldi, 0.0);
  const int ldh = kMaxArnoldi;
  launch_start_vector(c, L, c.opts.seed, V, s);
  double nrm = wnorm(c, L, V, s);
  if (nrm == 0.0) return 0.0;
  launch_axpby<double>(L.nloc, 1.0 / nrm, V, 0.0, V, s);
  int k = 0;
  double hmax = 0.0;
  for (int j = 0; j < m; ++j) {
    double *w = V + (j + 1) * ld;
    opA<double>(c, L, V + j * ld, L.d_t, s);
    opS<double>(c, L, L.d_t, w, s);
    // classical Gram-Schmidt, twice
    std::vector<double> h(j + 1, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
      launch_mdot(c, L.nloc, L.w64, j + 1, V, ld, w, c.dres, s);
      launch_mupdate(L.nloc, j + 1, V, ld, c.dres, w, -1.0, s);
      host_scalars(c, c.dres, (j + 1) * sizeof(double), s);
      for (int i = 0; i <= j; ++i) h[i] += c.hres[i];
    }
    double hn = wnorm(c, L, w, s);
    for (int i = 0; i <= j; ++i) {
      H[i * ldh + j] = h[i];
      hmax = std::max(hmax, std::fabs(h[i]));
    }
    H[(j + 1) * ldh + j] = hn;
    hmax = std::max(hmax, hn);
    k = j + 1;
    if (hn <= 1e-14 * hmax) break;
    launch_axpby<double>(L.nloc, 1.0 / hn, w, 0.0, w, s);
  }
  return hessenberg_max_abs_eig(H.data(), ldh, k);
}

// ---------------------------------------------------------------------------
static void setup(Ctx &c, const sem_mesh *m, void *ws, size_t bytes, hipStream_t s) {
  Arena A;
  A.base = static_cast<char *>(ws);
  A.cap = bytes;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) fail(SEM_EINVAL, "workspace must be 256-byte aligned");
  SetupScratch sc;
  layout(c, m, A, sc);
  SEM_HIP(hipHostMalloc((void **)&c.hres, 4096, hipHostMallocDefault));

  const int Ng = m->p_geom + 1;
  const int64_t E = c.lev[0].E;
  SEM_HIP(hipMemcpyAsync(sc.xyz, m->xyz, (size_t)E * Ng * Ng * Ng * 3 * sizeof(double),
                         hipMemcpyHostToDevice, s));
  SEM_HIP(hipMemsetAsync(sc.bad, 0, 64 * sizeof(int), s));
  SEM_HIP(hipMemsetAsync(c.counter, 0, 64 * sizeof(unsigned), s));
  launch_gll(m->p_geom, sc.xig, nullptr, s);

  for (int l = 0; l < c.nlev; ++l) {
    Level &L = c.lev[l];
    launch_gll(L.p, L.xi, L.wq, s);
    launch_dmat(L.p, L.xi, L.D64, L.D32, s);
    launch_interp(m->p_geom, L.p, sc.xig, L.xi, sc.Jg, nullptr, s);
    launch_level_coords(c, sc.xyz, m->p_geom, sc.Jg, L, s);
    launch_geom(c, L, sc.bad, s);
    launch_geom16(L, s);
    sc.gs.off = 0;
    build_gather_scatter(c, L, sc.gs, s);
    launch_weights(L, s);
    launch_diag(L, L.d_t, s);
    launch_gs<double>(L, L.d_t, s);
    launch_jacobi_inv(L.nloc, L.d_t, L.w64, L.dinv64, L.dinv32, s);
    if (L.boxlen) {
      launch_boxlen(c, L, s);
      launch_fdm_setup(c, L, s);
    }
  }
  for (int l = 0; l + 1 < c.nlev; ++l) {
    Level &F = c.lev[l], &C = c.lev[l + 1];
    launch_interp(C.p, F.p, C.xi, F.xi, F.J64, F.J32, s);
  }
  if (c.cs) {
    SEM_HIP(hipMemsetAsync(c.cs->counter, 0, 64 * sizeof(unsigned), s));
    coarse_setup(c, c.lev[c.nlev - 1], s);
  }
  int bad = 0;
  SEM_HIP(hipMemcpyAsync(&bad, sc.bad, sizeof(int), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  if (bad) fail(SEM_EGEOM, "an element has a non-positive Jacobian determinant");
  if (c.lowp) {
    for (int l = 0; l < c.nlev; ++l)
      if (c.lev[l].S16) {
        launch_fdm_mfma(c, c.lev[l], nullptr, nullptr, false, -1, s);  // pack S
        if (c.lev[l].A16) launch_fdm_mf16_pack(c.lev[l], s);
      }
  }

  if (c.opts.precond == SEM_PRECOND_PMG) {
    for (int l = 0; l + 1 < c.nlev; ++l) {
      Level &L = c.lev[l];
      double lt = c.opts.lambda_override[l] > 0 ? c.opts.lambda_override[l] : arnoldi(c, l, s);
      if (!(lt > 0) || !std::isfinite(lt)) fail(SEM_ENAN, "Arnoldi gave no usable lambda~");
      L.lam_tilde = lt;
      L.lmin = c.opts.lmin_fac * lt;
      L.lmax = c.opts.lmax_fac * lt;
      L.K = c.opts.cheb_order;
    }
  }
  SEM_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Krylov solvers (FP64 on the finest level)
// rref > 0: the residual test is ||r|| <= rtol * rref instead of rtol * ||r_0||
static int solve_cg(Ctx &c, const double *b, double *x, double rtol, int maxit, bool flexible,
                    sem_solve_info *info, hipStream_t s, double rref = 0.0) {
  Level &F = c.lev[0];
  const int64_t n = F.nloc;
  double *r = c.kr, *z = c.kz, *zo = c.kzold, *p = c.kp, *q = c.kq;
  opA<double>(c, F, x, q, s);
  launch_sub<double>(n, b, q, r, s);
  const double r0 = wnorm(c, F, r, s);
  info->r0_norm = r0;
  if (r0 == 0.0 || (rref > 0.0 && r0 <= rtol * rref)) {
    info->rel_res = info->true_rel_res = rref > 0.0 ? r0 / rref : 0.0;
    info->converged = 1;
    return 0;
  }
  const double den = rref > 0.0 ? rref : r0;
  int it = 0;
  double rel = 1.0;
  bool breakdown = false;
  const bool zf = z_in_f32(c);
  // Device scalars: (r, z) and (r, z_old) in two alternating pairs, (p, q) and
  // (r, r).  alpha and beta are formed on the device from them, so an iteration
  // reads back once: after the x, r update, (r, r) for the stopping test with
  // (p, q) and (r, z) for the breakdown and NaN checks.
  double *ds = c.dres + 2 * kMaxRestart + 32;
  double *const dpq = ds + 4, *const drr = ds + 5;
  int slot = 0;  // pair holding the current (r, z)
  auto rz_dots = [&](int nd, double *out) {
    if (zf) {
      launch_wdots_rz(c, n, F.w64, F.w32, r, F.f_x, nd == 2 ? c.fzo : nullptr, out, s);
    } else {
      const double *a[2] = {r, r}, *bb[2] = {z, zo};
      launch_wdots(c, n, F.w64, nd, a, bb, out, s, F.w32);
    }
  };
  while (it < maxit) {
    if (zf) {
      precondition_f32(c, r, s);
      launch_copy_cvt_f2d(n, F.f_x, p, s);
    } else {
      precondition(c, r, z, s);
      SEM_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    rz_dots(1, ds + 2 * slot);
    while (it < maxit) {
      XDefer xq;
      opA_dot(c, F, p, q, dpq, s, &xq);
      // x, r, (r, r) in one pass (and the V-cycle's FP32 copy of r on the mixed path)
      launch_fcg_xr(c, n, ds + 2 * slot, dpq, F.w64, p, q, x, r, drr, s, F.w32,
                    zf ? F.f_b : nullptr, xq);
      host_scalars(c, ds, 6 * sizeof(double), s);
      const double *h = c.hres;
      if (!std::isfinite(h[2 * slot]) || !std::isfinite(h[4]) || !std::isfinite(h[5]))
        fail(SEM_ENAN, "NaN/Inf in an inner product");
      if (!(h[4] > 0.0)) {  // exact breakdown: p = 0, the iterate is final (x, r unchanged)
        breakdown = true;
        break;
      }
      ++it;
      rel = std::sqrt(h[5]) / den;
      if (rel <= rtol) break;
      if (zf) {
        std::swap(F.f_x, c.fzo);  // the V-cycle writes the new z; the old one stays
        precondition_f32(c, r, s, true);
      } else {
        std::swap(z, zo);
        precondition(c, r, z, s);
      }
      slot ^= 1;
      rz_dots(flexible ? 2 : 1, ds + 2 * slot);
      if (zf)
        launch_zp<float>(n, F.f_x, ds + 2 * slot, ds + 2 * (slot ^ 1), flexible, p, s);
      else
        launch_zp<double>(n, z, ds + 2 * slot, ds + 2 * (slot ^ 1), flexible, p, s);
    }
    // true residual
    opA<double>(c, F, x, q, s);
    launch_sub<double>(n, b, q, r, s);
    double tr = wnorm(c, F, r, s) / den;
    info->rel_res = rel;
    info->true_rel_res = tr;
    if (tr <= rtol) {
      info->converged = 1;
      return it;
    }
    if (breakdown) break;
  }
  info->converged = 0;
  return it;
}

static int solve_fgmres(Ctx &c, const double *b, double *x, double rtol, int maxit,
                        sem_solve_info *info, hipStream_t s, double rref = 0.0) {
  Level &F = c.lev[0];
  const int64_t n = F.nloc;
  const int m = c.opts.gmres_restart;
  double *r = c.kr, *q = c.kq;
  double *V = c.gV, *Z = c.gZ;
  opA<double>(c, F, x, q, s);
  launch_sub<double>(n, b, q, r, s);
  const double r0 = wnorm(c, F, r, s);
  info->r0_norm = r0;
  if (r0 == 0.0 || (rref > 0.0 && r0 <= rtol * rref)) {
    info->rel_res = info->true_rel_res = rref > 0.0 ? r0 / rref : 0.0;
    info->converged = 1;
    return 0;
  }
  const double den = rref > 0.0 ? rref : r0;
  int it = 0;
  double rel = 1.0;
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (it < maxit) {
    double beta = wnorm(c, F, r, s);
    launch_axpby<double>(n, 1.0 / beta, r, 0.0, V, s);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0, jused = 0;
    for (j = 0; j < m; ++j) {
      double *vj = V + j * n, *w = V + (j + 1) * n, *zj = Z + j * n;
      precondition(c, vj, zj, s);
      opA<double>(c, F, zj, w, s);
      std::vector<double> h(j + 1, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        launch_mdot(c, n, F.w64, j + 1, V, n, w, c.dres, s);
        launch_mupdate(n, j + 1, V, n, c.dres, w, -1.0, s);
        host_scalars(c, c.dres, (j + 1) * sizeof(double), s);
        for (int i = 0; i <= j; ++i) h[i] += c.hres[i];
      }
      double hn = wnorm(c, F, w, s);
      // apply previous rotations to the new column, then a new one
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      double den = std::sqrt(h[j] * h[j] + hn * hn);
      cs[j] = den > 0 ? h[j] / den : 1.0;
      sn[j] = den > 0 ? hn / den : 0.0;
      h[j] = den;
      for (int i = 0; i <= j; ++i) H[i * m + j] = h[i];
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jused = j + 1;
      rel = std::fabs(g[j + 1]) / den;
      if (!std::isfinite(rel)) fail(SEM_ENAN, "NaN in FGMRES");
      if (rel <= rtol || it >= maxit || hn == 0.0) break;
      launch_axpby<double>(n, 1.0 / hn, w, 0.0, w, s);
    }
    // y = R^{-1} g, x += Z y
    for (int i = jused - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k = i + 1; k < jused; ++k) acc -= H[i * m + k] * y[k];
      y[i] = acc / H[i * m + i];
    }
    SEM_HIP(hipMemcpyAsync(c.dres, y.data(), jused * sizeof(double), hipMemcpyHostToDevice, s));
    launch_mupdate(n, jused, Z, n, c.dres, x, 1.0, s);
    opA<double>(c, F, x, q, s);
    launch_sub<double>(n, b, q, r, s);
    double tr = wnorm(c, F, r, s) / den;
    info->rel_res = rel;
    info->true_rel_res = tr;
    if (tr <= rtol) {
      info->converged = 1;
      return it;
    }
  }
  info->converged = 0;
  return it;
}

// Successive right sides (Sec. 3.2 / 4.2): start from the A-conjugate
// projection of b onto the prior solutions, x0 = sum_i (x_i, b) x_i with
// (x_i, A x_j) = delta_ij, so x0 is the A-norm best approximation of A^{-1} b in
// their span; stop at ||r|| <= rtol ||b||; then A-orthogonalise the correction
// x - x0 against the basis (classical Gram-Schmidt, two passes, using the
// stored A x_i) and append it.  A full basis restarts from the solution alone.
static int solve_projected(Ctx &c, const double *b, double *x, double rtol, int maxit,
                           sem_solve_info *info, hipStream_t s) {
  Level &F = c.lev[0];
  const int64_t n = F.nloc;
  const int L = c.nproj;
  double *X = c.projX, *AX = c.projAX, *w = c.projW, *Aw = c.projAW;
  const double nb = wnorm(c, F, b, s);
  launch_fill(n, 0.0, x, s);
  if (L > 0) {
    launch_mdot(c, n, F.w64, L, X, n, b, c.dres, s);  // alpha_i = (x_i, b)
    launch_mupdate(n, L, X, n, c.dres, x, 1.0, s);   // x0 = sum_i alpha_i x_i
  }
  launch_copy<double>(n, x, w, s);
  int it;
  if (c.opts.krylov == SEM_KRYLOV_FGMRES)
    it = solve_fgmres(c, b, x, rtol, maxit, info, s, nb > 0.0 ? nb : 1.0);
  else
    it = solve_cg(c, b, x, rtol, maxit, c.opts.krylov == SEM_KRYLOV_FCG, info, s,
                  nb > 0.0 ? nb : 1.0);
  // the new direction: x - x0, or the whole solution when the basis is full
  int Lb = L;
  if (L == c.opts.proj_max) {
    Lb = 0;
    launch_copy<double>(n, x, w, s);
  } else {
    launch_axpby<double>(n, 1.0, x, -1.0, w, s);
  }
  opA<double>(c, F, w, Aw, s);
  const double *pw[1] = {w}, *paw[1] = {Aw};
  double n0;
  dots(c, F, 1, pw, paw, &n0, s);
  for (int pass = 0; pass < 2 && Lb > 0; ++pass) {
    launch_mdot(c, n, F.w64, Lb, X, n, Aw, c.dres, s);  // beta_i = (x_i, A w)
    launch_mupdate(n, Lb, X, n, c.dres, w, -1.0, s);
    launch_mupdate(n, Lb, AX, n, c.dres, Aw, -1.0, s);
  }
  double nn;
  dots(c, F, 1, pw, paw, &nn, s);
  if (nn > 0.0 && nn > 1e-20 * n0) {  // keep only a direction the basis does not hold
    const double inv = 1.0 / std::sqrt(nn);
    launch_axpby<double>(n, inv, w, 0.0, X + (int64_t)Lb * n, s);
    launch_axpby<double>(n, inv, Aw, 0.0, AX + (int64_t)Lb * n, s);
    ++Lb;
  }
  c.nproj = Lb;
  return it;
}

// entry points used by the batched driver (batch.hip)
void batch_opA(const Ctx &c, const Level &L, const double *u, double *Au, hipStream_t s, int nv) {
  opA<double>(c, L, u, Au, s, nv);
}
void batch_precondition(Ctx &c, const double *r, double *z, hipStream_t s, int nv) {
  precondition(c, r, z, s, nv);
}
double batch_wnorm2(Ctx &c, const double *a, const double *b, hipStream_t s) {
  const double *pa[1] = {a}, *pb[1] = {b};
  double v;
  dots(c, c.lev[0], 1, pa, pb, &v, s);
  return v;
}

static Level &level_of(sem_ctx *ctx, int level) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) fail(SEM_EINVAL, "null context");
  if (level < 0 || level >= c->nlev) fail(SEM_EINVAL, "level out of range");
  return c->lev[level];
}

}  // namespace sem

using namespace sem;

struct sem_ctx : public sem::Ctx {};

// ---------------------------------------------------------------------------
// Reduction scratch of sem_solve_static: a file-scope device array instead of
// the context's workspace.  Layout in doubles: block partials of every
// reduction [kRedBlocks][8], reduction results (FGMRES and projection
// coefficients included), the device scalars of the Krylov recurrence, the
// last-block ticket counters, then the finest level's element shares of
// (p, A p).  Each device holds its own copy, at its own address, for the life
// of the process.
constexpr size_t kStPartials = 0;
constexpr size_t kStDres = kStPartials + (size_t)kRedBlocks * 8;
constexpr size_t kStDsc = kStDres + 256;
constexpr size_t kStCounter = kStDsc + 32;
constexpr size_t kStDot = kStCounter + 32;
constexpr size_t kStaticDoubles = 65536;  // 512 KiB
constexpr int64_t kStaticMaxElements = (int64_t)(kStaticDoubles - kStDot);
static_assert(2 * kMaxRestart + 64 <= 256, "reduction results exceed their slot");
static_assert(sizeof(DevScalars) <= 32 * sizeof(double), "device scalars exceed their slot");
static_assert(64 * sizeof(unsigned) <= 32 * sizeof(double), "counters exceed their slot");

static __device__ __align__(256) double scratch[kStaticDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Device address of the current device's copy of `scratch` (looked up once per
// device; host code must never pass the symbol itself to a kernel).
static double *static_scratch() {
  int dev = 0;
  SEM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(SEM_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    SEM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(SEM_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[dev];
}

// Points the context's reduction scratch at the static array for the scope
// of one call, and back afterwards (also when the call fails).
struct StaticScratchScope {
  Ctx &c;
  double *partials, *dres, *dot;
  unsigned *counter;
  DevScalars *dsc;
  StaticScratchScope(Ctx &cx, hipStream_t s) : c(cx) {
    partials = c.partials;
    dres = c.dres;
    dsc = c.dsc;
    counter = c.counter;
    dot = c.lev[0].dotpart;
    if (c.lev[0].E > kStaticMaxElements)
      fail(SEM_EINVAL, "sem_solve_static: the finest level has " + std::to_string(c.lev[0].E) +
                           " elements, more than the static scratch holds (" +
                           std::to_string(kStaticMaxElements) + ")");
    double *base = static_scratch();
    c.partials = base + kStPartials;
    c.dres = base + kStDres;
    c.dsc = reinterpret_cast<DevScalars *>(base + kStDsc);
    c.counter = reinterpret_cast<unsigned *>(base + kStCounter);
    if (dot) c.lev[0].dotpart = base + kStDot;
    // the last-block tickets must start at zero (a fill kernel: no memset
    // node, should the caller capture the call into a graph)
    launch_fill(32, 0.0, base + kStCounter, s);
  }
  ~StaticScratchScope() {
    c.partials = partials;
    c.dres = dres;
    c.dsc = dsc;
    c.counter = counter;
    c.lev[0].dotpart = dot;
  }
};

extern "C" {

void sem_default_opts(sem_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nlevels = 3;
  o->p_levels[0] = 7;
  o->p_levels[1] = 3;
  o->p_levels[2] = 1;
  o->precond = SEM_PRECOND_PMG;
  o->smoother = SEM_SMOOTH_JACOBI;
  o->cheb_order = 2;
  o->lmin_fac = 0.1;
  o->lmax_fac = 1.1;
  o->arnoldi_steps = 10;
  o->seed = 0;
  o->smoother_prec = SEM_F64;
  o->fdm_prec = SEM_F64;
  o->krylov = SEM_KRYLOV_FCG;
  o->gmres_restart = 20;
  o->coarse_tol = 1e-10;
  o->coarse_maxit = 2000;
  o->ax_variant = -1;
  o->batch_rhs = 0;
  o->coarse_solver = -1;
  o->proj_max = 0;
  o->geom_prec = SEM_F32;
}

const char *sem_last_error(void) { return g_last_error.c_str(); }

sem_status sem_plan(const sem_mesh *mesh, int32_t p, const int8_t bc[6], const sem_opts *opts,
                    size_t *bytes) {
  return guarded([&] {
    if (!bytes) fail(SEM_EINVAL, "null size pointer");
    validate(mesh, p, bc, opts);
    Ctx c;
    init_ctx(c, mesh, p, bc, opts);
    Arena A;
    SetupScratch sc;
    layout(c, mesh, A, sc);
    *bytes = A.off + 256;
  });
}

sem_status sem_setup(const sem_mesh *mesh, int32_t p, const int8_t bc[6], const sem_opts *opts,
                     void *ws, size_t bytes, void *stream, sem_ctx **out) {
  sem_ctx *c = nullptr;
  sem_status st = guarded([&] {
    if (!out || !ws) fail(SEM_EINVAL, "null workspace or output pointer");
    *out = nullptr;
    validate(mesh, p, bc, opts);
    if (!mesh->xyz) fail(SEM_EINVAL, "null coordinates");
    c = new sem_ctx();
    init_ctx(*c, mesh, p, bc, opts);
    setup(*c, mesh, ws, bytes, as_stream(stream));
    (void)static_scratch();  // this device's address of the sem_solve_static scratch
    *out = c;
  });
  if (st != SEM_OK && c) {
    if (c->cs) coarse_release(*c->cs);
    if (c->hres) (void)hipHostFree(c->hres);
    delete c->prof;
    delete c;
  }
  return st;
}

sem_status sem_destroy(sem_ctx *ctx) {
  return guarded([&] {
    if (!ctx) return;
    if (ctx->cs) coarse_release(*ctx->cs);
    if (ctx->hres) SEM_HIP(hipHostFree(ctx->hres));
    delete ctx->prof;
    delete ctx;
  });
}

sem_status sem_profile(sem_ctx *ctx, int32_t enable) {
  return guarded([&] {
    if (!ctx) fail(SEM_EINVAL, "null context");
    if (enable < 0) fail(SEM_EINVAL, "profile: negative class mask");
    if (!ctx->prof) ctx->prof = new Profiler();
    ctx->prof->reset();
    ctx->prof->on = enable != 0;
    ctx->prof->kinds = enable == 1 ? ~0u : (unsigned)enable >> 1;
  });
}

sem_status sem_profile_read(sem_ctx *ctx, double *total_ms, int64_t *launches) {
  return guarded([&] {
    if (!ctx || !total_ms || !launches) fail(SEM_EINVAL, "null argument");
    for (int k = 0; k < SEM_PROF_COUNT; ++k) {
      total_ms[k] = 0.0;
      launches[k] = 0;
    }
    if (!ctx->prof) return;
    for (auto &r : ctx->prof->recs) {
      SEM_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      SEM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      total_ms[r.kind] += ms;
      launches[r.kind] += 1;
    }
  });
}

sem_status sem_level_info(const sem_ctx *ctx, int32_t level, sem_level_desc *out) {
  return guarded([&] {
    if (!out) fail(SEM_EINVAL, "null output");
    const Level &L = level_of(const_cast<sem_ctx *>(ctx), level);
    out->p = L.p;
    out->N = L.N;
    out->E = L.E;
    out->nlocal = L.nloc;
    out->nglobal = L.nglob;
    out->nshared = L.nseg;
    out->nmembers = L.nperm;
    out->lmin = L.lmin;
    out->lmax = L.lmax;
  });
}

sem_status sem_gll(int32_t p, double *nodes, double *weights, void *stream) {
  return guarded([&] {
    if (p < 1 || p > 15) fail(SEM_EINVAL, "p must be in [1, 15]");
    if (!nodes) fail(SEM_EINVAL, "null nodes");
    launch_gll(p, nodes, weights, as_stream(stream));
  });
}

sem_status sem_coords(const sem_ctx *ctx, int32_t level, double *xyz, void *stream) {
  return guarded([&] {
    const Level &L = level_of(const_cast<sem_ctx *>(ctx), level);
    if (!xyz) fail(SEM_EINVAL, "null output");
    SEM_HIP(hipMemcpyAsync(xyz, L.X, 3 * L.nloc * sizeof(double), hipMemcpyDeviceToDevice,
                           as_stream(stream)));
  });
}

sem_status sem_gather(const sem_ctx *ctx, int32_t level, const double *ug, double *ul,
                      void *stream) {
  return guarded([&] {
    const Level &L = level_of(const_cast<sem_ctx *>(ctx), level);
    if (!ug || !ul) fail(SEM_EINVAL, "null vector");
    launch_gather(*ctx, L, ug, ul, as_stream(stream));
  });
}

sem_status sem_rhs(sem_ctx *ctx, const double *f, double *b, void *stream) {
  return guarded([&] {
    Level &L = level_of(ctx, 0);
    if (!f || !b) fail(SEM_EINVAL, "null vector");
    launch_rhs(L, f, b, as_stream(stream));
    launch_gs<double>(L, b, as_stream(stream));
  });
}

sem_status sem_apply_A(sem_ctx *ctx, int32_t level, int32_t prec, const void *u, void *Au,
                       void *stream) {
  return guarded([&] {
    Level &L = level_of(ctx, level);
    if (!u || !Au || u == Au) fail(SEM_EINVAL, "null or aliased vectors");
    hipStream_t s = as_stream(stream);
    if (prec == SEM_F64)
      opA<double>(*ctx, L, (const double *)u, (double *)Au, s);
    else if (prec == SEM_F32)
      opA<float>(*ctx, L, (const float *)u, (float *)Au, s);
    else
      fail(SEM_EINVAL, "prec must be SEM_F64 or SEM_F32");
  });
}

sem_status sem_apply_S(sem_ctx *ctx, int32_t level, int32_t prec, const void *r, void *z,
                       void *stream) {
  return guarded([&] {
    Level &L = level_of(ctx, level);
    if (!r || !z || r == z) fail(SEM_EINVAL, "null or aliased vectors");
    hipStream_t s = as_stream(stream);
    if (prec == SEM_F64)
      opS<double>(*ctx, L, (const double *)r, (double *)z, s);
    else if (prec == SEM_F32)
      opS<float>(*ctx, L, (const float *)r, (float *)z, s);
    else
      fail(SEM_EINVAL, "prec must be SEM_F64 or SEM_F32");
  });
}

sem_status sem_smooth(sem_ctx *ctx, int32_t level, int32_t prec, const void *b, void *x,
                      void *stream) {
  return guarded([&] {
    Level &L = level_of(ctx, level);
    if (L.coarse || ctx->opts.precond != SEM_PRECOND_PMG)
      fail(SEM_EINVAL, "level has no smoother (coarsest level or Jacobi preconditioner)");
    if (!b || !x) fail(SEM_EINVAL, "null vector");
    hipStream_t s = as_stream(stream);
    if (prec == SEM_F64)
      chebyshev<double>(*ctx, L, (const double *)b, (double *)x, false, s);
    else if (prec == SEM_F32)
      chebyshev<float>(*ctx, L, (const float *)b, (float *)x, false, s);
    else
      fail(SEM_EINVAL, "prec must be SEM_F64 or SEM_F32");
  });
}

sem_status sem_prolong(sem_ctx *ctx, int32_t level, int32_t prec, const void *xc, void *xf,
                       void *stream) {
  return guarded([&] {
    Level &F = level_of(ctx, level);
    Level &C = level_of(ctx, level + 1);
    if (!xc || !xf) fail(SEM_EINVAL, "null vector");
    hipStream_t s = as_stream(stream);
    if (prec == SEM_F64)
      launch_prolong<double>(F, C, (const double *)xc, (double *)xf, s);
    else if (prec == SEM_F32)
      launch_prolong<float>(F, C, (const float *)xc, (float *)xf, s);
    else
      fail(SEM_EINVAL, "prec must be SEM_F64 or SEM_F32");
  });
}

sem_status sem_restrict(sem_ctx *ctx, int32_t level, int32_t prec, const void *rf, void *rc,
                        void *stream) {
  return guarded([&] {
    Level &F = level_of(ctx, level);
    Level &C = level_of(ctx, level + 1);
    if (!rf || !rc) fail(SEM_EINVAL, "null vector");
    hipStream_t s = as_stream(stream);
    if (prec == SEM_F64) {
      launch_restrict<double>(F, C, (const double *)rf, (double *)rc, s);
      launch_gs<double>(C, (double *)rc, s);
    } else if (prec == SEM_F32) {
      if (!F.w32) fail(SEM_EINVAL, "FP32 weights were not built");
      launch_restrict<float>(F, C, (const float *)rf, (float *)rc, s);
      launch_gs<float>(C, (float *)rc, s);
    } else {
      fail(SEM_EINVAL, "prec must be SEM_F64 or SEM_F32");
    }
  });
}

sem_status sem_vcycle(sem_ctx *ctx, const double *r, double *z, void *stream) {
  return guarded([&] {
    if (!ctx) fail(SEM_EINVAL, "null context");
    if (!r || !z) fail(SEM_EINVAL, "null vector");
    precondition(*ctx, r, z, as_stream(stream));
  });
}

static sem_status solve_entry(sem_ctx *ctx, const double *b, double *x, double rtol, int32_t maxit,
                              sem_solve_info *info, void *stream, bool static_scratch_only) {
  sem_solve_info local{};
  sem_solve_info *inf = info ? info : &local;
  std::memset(inf, 0, sizeof(*inf));
  bool noconv = false;
  sem_status st = guarded([&] {
    if (!ctx) fail(SEM_EINVAL, "null context");
    if (!b || !x) fail(SEM_EINVAL, "null vector");
    if (!(rtol > 0) || maxit < 0) fail(SEM_EINVAL, "rtol must be > 0 and maxit >= 0");
    hipStream_t s = as_stream(stream);
    std::unique_ptr<StaticScratchScope> scope;
    if (static_scratch_only) scope.reset(new StaticScratchScope(*ctx, s));
    for (int l = 0; l < ctx->nlev; ++l) inf->lambda_tilde[l] = ctx->lev[l].lam_tilde;
    int it;
    if (ctx->opts.proj_max > 0)
      it = solve_projected(*ctx, b, x, rtol, maxit, inf, s);
    else if (ctx->opts.krylov == SEM_KRYLOV_FGMRES)
      it = solve_fgmres(*ctx, b, x, rtol, maxit, inf, s);
    else
      it = solve_cg(*ctx, b, x, rtol, maxit, ctx->opts.krylov == SEM_KRYLOV_FCG, inf, s);
    inf->iters = it;
    inf->coarse_iters = ctx->last_coarse_iters;
    SEM_HIP(hipStreamSynchronize(s));
    noconv = !inf->converged;
  });
  if (st == SEM_OK && noconv) {
    g_last_error = "no convergence within maxit iterations";
    return SEM_ENOCONV;
  }
  return st;
}

sem_status sem_solve(sem_ctx *ctx, const double *b, double *x, double rtol, int32_t maxit,
                     sem_solve_info *info, void *stream) {
  return solve_entry(ctx, b, x, rtol, maxit, info, stream, false);
}

sem_status sem_solve_static(sem_ctx *ctx, const double *b, double *x, double rtol, int32_t maxit,
                            sem_solve_info *info, void *stream) {
  return solve_entry(ctx, b, x, rtol, maxit, info, stream, true);
}

sem_status sem_projection_reset(sem_ctx *ctx) {
  return guarded([&] {
    if (!ctx) fail(SEM_EINVAL, "null context");
    ctx->nproj = 0;
  });
}

}  // extern "C"
