// C ABI of the HOPU convection library: context, argument checks, dispatch
// by (dim, k), the PCG mass solve and the substep driver.
#include "../../include/hopu.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "aux.hpp"
#include "host_tables.hpp"
#include "kernels.hpp"
#include "proj.hpp"
#include "stokes.hpp"
#include "launch.hpp"
#include "launch_events.hpp"
#include "vec.hpp"

// A named range around an entry point's host work and launches, for
// rocprofv3's marker trace (roctx; a host call, no stream operation).
struct RocRange {
  explicit RocRange(const char* name) { roctxRangePushA(name); }
  ~RocRange() { roctxRangePop(); }
  RocRange(const RocRange&) = delete;
  RocRange& operator=(const RocRange&) = delete;
};

using namespace hopu;

struct hopu_ctx_s {
  int dim = 0, k = 0;
  Sizes sz;
  FragDims fd;
  hipStream_t stream = nullptr;
  int64_t n_dof = 0;
  MeshData mesh;
  Batches bat;
  DevMesh dm;
  DevTables<double> tb64;
  DevTables<float> tb32;
  DevTables<BfPack<2>> tbb2;  // split-BF16 tables (hi/lo)
  DevTables<BfPack<3>> tbb3;  // (hi/mid/lo)
  const double *mass_in = nullptr, *mass_out = nullptr, *prec_in = nullptr, *prec_out = nullptr;
  const float *prec_in32 = nullptr, *prec_out32 = nullptr;  // FP32 preconditioner tables
  const double* vol_dV64 = nullptr;
  const double *psi_n64 = nullptr, *psi_n32 = nullptr;  // u.n tables for the f64 / f32 row maps
  double* xyz = nullptr;
  // workspaces
  double* m64 = nullptr;
  float* m32 = nullptr;
  double* mu64 = nullptr;   // modal coefficients of the adjoint argument
  float* mu32 = nullptr;
  double* slot = nullptr;
  double* part = nullptr;   // partial sums (max(NPART, nb, waves))
  double* part2 = nullptr;  // partial sums of the vector updates (2 NPART)
  int64_t npart = 0;
  double *r = nullptr, *z = nullptr, *q = nullptr, *w = nullptr, *rc = nullptr;
  // PCG search directions p_i, ring of nph vectors, with their alpha_i: the
  // solution update x += sum alpha_i p_i is made in one pass at the end (and
  // whenever the ring is full) instead of a read and write of x per iteration
  double* phist = nullptr;
  double* ahist = nullptr;
  int nph = 0;
  // projection step (tables at create; workspace on the first hopu_project)
  const double *proj_b = nullptr, *proj_bt = nullptr, *proj_kab = nullptr;
  const int32_t* mfid = nullptr;
  double *ainv = nullptr, *ph = nullptr, *pr = nullptr, *pfs = nullptr;
  double *pph = nullptr, *paht = nullptr;  // its CG's direction ring and alphas (as in the PCG)
  int npph = 0;
  bool proj_ready = false;
  double* stage = nullptr;  // 16-byte aligned copy of a mass-kernel input that is not
  double* wh[3] = {nullptr, nullptr, nullptr};  // previous substep solutions (newest first)
  int nwh = 0;              // how many of them a continuing hopu_substeps may use
  bool carry_warm = false;  // hopu_set_warm_start
  double* sc = nullptr;
  int* flag = nullptr;      // [0] converged, [1] iterations
  unsigned long long* nbad = nullptr;  // hopu_count_nonfinite's counter
  int* hflag = nullptr;     // pinned host copy
  std::vector<void*> allocs;
  DualBasis eval_db;              // reference dual basis (evaluation at given points)
  double* eval_scratch = nullptr;  // this device's copy of the evaluation scratch array
  int lglob = -1;
  const int8_t* lfac = nullptr;
  double rtol = 1e-13;
  int max_it = 500, check_every = 4;
  std::string err;
  // per-kernel timing with HIP events (hopu_profile_*)
  int last_its = 0;
  // adaptive HOPU order
  int8_t* own_lfac = nullptr;   // [F] facet orders owned by the context
  double* eta_nd = nullptr;     // [F][2] jump-indicator numerator/denominator
  int adapt_every = 0;
  double thr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  bool prof = false;
  int prof_stride = 1;                  // time every prof_stride-th launch of each kind
  int64_t prof_count[8] = {};           // launches seen per kind
  bool prof_armed = false;
  std::vector<hipEvent_t> events;       // pool, pairs
  std::vector<int> ev_kind;             // kernel id per used pair
  size_t ev_used = 0;
  // implicit Stokes step (tables and workspaces on the first hopu_stokes_setup)
  StokesDims st_sd;
  StokesDev st_dv{};
  bool st_alloc = false, st_ready = false, st_fp32 = false;
  double st_nu = 0.0, st_dt = 0.0;
  double *st_S = nullptr, *st_Sinv = nullptr, *st_slot = nullptr;
  double *st_r = nullptr, *st_z = nullptr, *st_p = nullptr, *st_q = nullptr, *st_b = nullptr;
  double *st_mu = nullptr, *st_conv = nullptr, *st_part = nullptr;
  int* st_bad = nullptr;
};

enum { PROF_ELEM = 0, PROF_MASS = 1, PROF_PREC = 2, PROF_MODAL = 3, PROF_VJP = 4, PROF_PLAIN = 5, PROF_STOKES_S = 6,
       PROF_STOKES_C = 7, PROF_N = 8 };
static_assert(PROF_N <= 8, "prof_count holds 8 kinds");

namespace hopu {
static thread_local LaunchEvents tl_events;
static thread_local bool tl_armed = false;
LaunchEvents* take_launch_events() {
  if (!tl_armed) return nullptr;
  tl_armed = false;
  return &tl_events;
}
void arm_launch_events(hipEvent_t start, hipEvent_t stop) {
  tl_events = LaunchEvents{start, stop};
  tl_armed = true;
}
void disarm_launch_events() { tl_armed = false; }
}  // namespace hopu

// the next launch through HOPU_LAUNCH records its dispatch into a pair
static void prof_begin(hopu_ctx ctx, int kind) {
  if (!ctx->prof || 2 * (ctx->ev_used + 1) > ctx->events.size()) return;
  if (ctx->prof_count[kind]++ % ctx->prof_stride != 0) return;
  arm_launch_events(ctx->events[2 * ctx->ev_used], ctx->events[2 * ctx->ev_used + 1]);
  ctx->ev_kind[ctx->ev_used] = kind;
  ctx->prof_armed = true;
}
static void prof_end(hopu_ctx ctx) {
  if (!ctx->prof_armed) return;
  disarm_launch_events();
  ++ctx->ev_used;
  ctx->prof_armed = false;
}

static std::string g_create_err;

#define HCHECK(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);         \
      return HOPU_EHIP;                                                     \
    }                                                                       \
  } while (0)

template <typename T>
static hopu_status dev_alloc(hopu_ctx ctx, T** p, size_t count) {
  if (count == 0) count = 1;
  const char* fail = std::getenv("HOPU_TEST_FAIL_ALLOC");
  if (fail && std::atoi(fail) == 1) {
    ctx->err = "device allocation refused (HOPU_TEST_FAIL_ALLOC)";
    return HOPU_ENOMEM;
  }
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess) {
    ctx->err = std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) + " bytes: " + hipGetErrorString(e);
    return HOPU_ENOMEM;
  }
  ctx->allocs.push_back(v);
  *p = (T*)v;
  return HOPU_OK;
}

template <typename T>
static hopu_status upload(hopu_ctx ctx, const T** dst, const std::vector<T>& src) {
  T* d = nullptr;
  hopu_status st = dev_alloc(ctx, &d, src.size());
  if (st) return st;
  if (!src.empty()) HCHECK(hipMemcpyAsync(d, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  *dst = d;
  return HOPU_OK;
}

static std::vector<float> to_f32(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

// the split-BF16 element-kernel tables with NS terms, from the FP32-layout set
template <int NS>
static hopu_status upload_bf16(hopu_ctx ctx, const FragTables& f32, int ns, DevTables<BfPack<NS>>& t,
                               const double* dual64, const double* wv, const double* wf, const int* pdeg) {
  if (ns != NS) return HOPU_EINVAL;
  BfTables b;
  make_bf16_tables(f32, ctx->sz, NS, b);
  auto up = [&](const BfPack<NS>** d, const std::vector<uint16_t>& v) {
    const uint16_t* p = nullptr;
    hopu_status st = upload(ctx, &p, v);
    *d = reinterpret_cast<const BfPack<NS>*>(p);
    return st;
  };
  hopu_status st;
  if ((st = up(&t.vol_V, b.vol_V)) || (st = up(&t.vol_dVT, b.vol_dVT)) || (st = up(&t.fac_Tr, b.fac_Tr)) ||
      (st = up(&t.fac_TrT, b.fac_TrT)) || (st = up(&t.fac_K, b.fac_K)) || (st = up(&t.fac_Psi, b.fac_Psi)) ||
      (st = up(&t.fac_PsiT, b.fac_PsiT)) || (st = up(&t.fac_KT, b.fac_KT)) || (st = up(&t.vol_dV, b.vol_dV)) ||
      (st = up(&t.vol_VT, b.vol_VT)))
    return st;
  t.modal = nullptr;  // the modal and dual transforms run in FP64
  t.dual = nullptr;
  t.dual64 = dual64;
  t.wv = wv;
  t.wf = wf;
  t.psi_deg = pdeg;
  return HOPU_OK;
}

#define DISPATCH(DIM, K, ...)                              \
  switch ((DIM) * 10 + (K)) {                               \
    case 21: { constexpr int D = 2, KK = 1; __VA_ARGS__; } break;  \
    case 22: { constexpr int D = 2, KK = 2; __VA_ARGS__; } break;  \
    case 23: { constexpr int D = 2, KK = 3; __VA_ARGS__; } break;  \
    case 24: { constexpr int D = 2, KK = 4; __VA_ARGS__; } break;  \
    case 31: { constexpr int D = 3, KK = 1; __VA_ARGS__; } break;  \
    case 32: { constexpr int D = 3, KK = 2; __VA_ARGS__; } break;  \
    case 33: { constexpr int D = 3, KK = 3; __VA_ARGS__; } break;  \
    case 34: { constexpr int D = 3, KK = 4; __VA_ARGS__; } break;  \
    case 35: { constexpr int D = 3, KK = 5; __VA_ARGS__; } break;  \
    default: break;                                         \
  }

static bool supported(int dim, int k) { return (dim == 2 && k >= 1 && k <= 4) || (dim == 3 && k >= 1 && k <= 5); }

static hopu_status fail(hopu_ctx ctx, hopu_status st, const std::string& msg) {
  ctx->err = msg;
  return st;
}

static void refresh_dm(hopu_ctx ctx) {
  ctx->dm.lfac = ctx->lfac;
  ctx->dm.lglob = ctx->lglob;
}

// Scratch of the allocation-free evaluation (hopu_eval_noalloc): the basis
// table at the caller's points, one copy per GPU for the life of the
// process, shared by every context on that GPU.  Host code reaches it only
// through the address hipGetSymbolAddress gives for each device (the name
// itself is a host-side stand-in).
static constexpr int64_t EVAL_SCRATCH_DOUBLES = 1 << 17;  // 1 MiB
static __device__ __align__(256) double scratch[EVAL_SCRATCH_DOUBLES];
static constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up once per device.
static hopu_status scratch_address(double** out, std::string& err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { err = std::string("hipGetDevice: ") + hipGetErrorString(e); return HOPU_EHIP; }
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) { err = "device index beyond the scratch table"; return HOPU_EUNSUPPORTED; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return HOPU_EHIP;
    }
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return HOPU_OK;
}

extern "C" hopu_status hopu_create(hopu_ctx* out, int dim, int k, int64_t n_elems, const int64_t* elem_vid,
                                   const double* elem_xyz, void* hip_stream) {
  if (!out) { g_create_err = "out is NULL"; return HOPU_EINVAL; }
  *out = nullptr;
  if (dim != 2 && dim != 3) { g_create_err = "dim must be 2 or 3"; return HOPU_EINVAL; }
  if (k < 1 || k > 6) { g_create_err = "k must be in 1..6"; return HOPU_EINVAL; }
  if (!supported(dim, k)) { g_create_err = "order not built into this library (3D k<=5, 2D k<=4)"; return HOPU_EUNSUPPORTED; }
  if (n_elems <= 0 || !elem_vid || !elem_xyz) { g_create_err = "empty mesh or NULL mesh arrays"; return HOPU_EINVAL; }
  if (n_elems > (int64_t)INT32_MAX / 2) { g_create_err = "too many elements"; return HOPU_EINVAL; }
  hopu_ctx ctx = new hopu_ctx_s();
  ctx->dim = dim;
  ctx->k = k;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->sz = make_sizes(dim, k);
  ctx->fd = frag_dims(ctx->sz);
  ctx->lglob = k - 1;
  std::string err;
  if (!build_mesh(dim, n_elems, elem_vid, elem_xyz, ctx->mesh, err)) {
    g_create_err = err;
    delete ctx;
    return HOPU_EMESH;
  }
  // |det J|^{(d-1)/d} for the interior DoF scaling
  for (int64_t e = 0; e < n_elems; ++e) {
    double* g = &ctx->mesh.geo[e * GEO_STRIDE];
    long double ad = fabsl((long double)g[GEO_DET]);
    g[GEO_SI] = (double)(dim == 2 ? sqrtl(ad) : powl(cbrtl(ad), 2.0L));
  }
  make_batches(ctx->mesh, ctx->bat);
  if (!make_dual_basis(dim, k, ctx->eval_db, err)) {
    g_create_err = err;
    delete ctx;
    return HOPU_EINVAL;
  }
  RefTables rt;
  if (!make_ref_tables(dim, k, rt, err)) {
    g_create_err = err;
    delete ctx;
    return HOPU_EINVAL;
  }
  FragTables f64, f32;
  make_frag_tables(rt, ROWMAP_F64, f64);
  make_frag_tables(rt, ROWMAP_F32, f32);
  const Sizes& s = ctx->sz;
  ctx->n_dof = ctx->mesh.F * s.nf + n_elems * s.nint;
  hopu_status st = HOPU_OK;
#define TRY(x)                         \
  do {                                 \
    st = (x);                          \
    if (st) goto fail_create;          \
  } while (0)
  {
    const double* dgeo;
    const int32_t *dfid, *dnbr, *dfe, *dbe, *dbs;
    const int8_t* dfl;
    TRY(upload(ctx, &dgeo, ctx->mesh.geo));
    TRY(upload(ctx, &dfid, ctx->mesh.fid));
    TRY(upload(ctx, &dnbr, ctx->mesh.nbr));
    TRY(upload(ctx, &dfe, ctx->mesh.facet_elem));
    TRY(upload(ctx, &dfl, ctx->mesh.facet_local));
    const int8_t* dfs;
    {
      std::vector<int8_t> fside((size_t)n_elems * (ctx->dim + 1), 0);
      for (int64_t F = 0; F < ctx->mesh.F; ++F)
        fside[(size_t)ctx->mesh.facet_elem[2 * F + 1] * (ctx->dim + 1) + ctx->mesh.facet_local[2 * F + 1]] = 1;
      TRY(upload(ctx, &dfs, fside));
    }
    TRY(upload(ctx, &dbe, ctx->bat.elem));
    TRY(upload(ctx, &dbs, ctx->bat.sig));
    const double* dxyz;
    TRY(upload(ctx, &dxyz, ctx->mesh.xyz));
    ctx->xyz = (double*)dxyz;
    ctx->dm = DevMesh{dgeo, dfid, dnbr, dfe, dfl, dfs, dbe, dbs, nullptr, n_elems, ctx->mesh.F, ctx->bat.nb, ctx->lglob};
    // tables
    const double *wv, *wf;
    const int* pdeg;
    TRY(upload(ctx, &wv, rt.wv));
    TRY(upload(ctx, &wf, rt.wf));
    TRY(upload(ctx, &pdeg, rt.psi_deg));
    auto up64 = [&](const double** d, const std::vector<double>& v) { return upload(ctx, d, v); };
    auto up32 = [&](const float** d, const std::vector<double>& v) { return upload(ctx, d, to_f32(v)); };
    DevTables<double>& a = ctx->tb64;
    DevTables<float>& b = ctx->tb32;
    TRY(up64(&a.modal, f64.modal));  // (the modal transform is FP64 in every form)
    b.modal = nullptr;
    TRY(up64(&a.vol_V, f64.vol_V)); TRY(up32(&b.vol_V, f32.vol_V));
    TRY(up64(&a.vol_dVT, f64.vol_dVT)); TRY(up32(&b.vol_dVT, f32.vol_dVT));
    TRY(up64(&a.vol_dV, f64.vol_dV)); TRY(up32(&b.vol_dV, f32.vol_dV));
    TRY(up64(&a.vol_VT, f64.vol_VT)); TRY(up32(&b.vol_VT, f32.vol_VT));
    TRY(up64(&a.fac_Tr, f64.fac_Tr)); TRY(up32(&b.fac_Tr, f32.fac_Tr));
    TRY(up64(&a.fac_TrT, f64.fac_TrT)); TRY(up32(&b.fac_TrT, f32.fac_TrT));
    TRY(up64(&a.fac_K, f64.fac_K)); TRY(up32(&b.fac_K, f32.fac_K));
    TRY(up64(&a.fac_Psi, f64.fac_Psi)); TRY(up32(&b.fac_Psi, f32.fac_Psi));
    TRY(up64(&a.fac_PsiT, f64.fac_PsiT)); TRY(up32(&b.fac_PsiT, f32.fac_PsiT));
    TRY(up64(&a.fac_KT, f64.fac_KT)); TRY(up32(&b.fac_KT, f32.fac_KT));
    // the dual transform is FP64 in every form; the reduced forms' table keeps
    // their K order
    TRY(up64(&a.dual, f64.dual)); TRY(up64(&b.dual64, f32.dual));
    a.dual64 = nullptr;
    b.dual = nullptr;
    a.wv = b.wv = wv;
    a.wf = b.wf = wf;
    a.psi_deg = b.psi_deg = pdeg;
    TRY(upload_bf16(ctx, f32, 2, ctx->tbb2, b.dual64, wv, wf, pdeg));
    TRY(upload_bf16(ctx, f32, 3, ctx->tbb3, b.dual64, wv, wf, pdeg));
    TRY(up64(&ctx->psi_n64, f64.psi_n));
    TRY(up64(&ctx->psi_n32, f32.psi_n));
    TRY(up64(&ctx->mass_in, f64.mass_in));
    TRY(up64(&ctx->mass_out, f64.mass_out));
    TRY(up64(&ctx->prec_in, f64.prec_in));
    TRY(up64(&ctx->prec_out, f64.prec_out));
    TRY(up32(&ctx->prec_in32, f32.prec_in));
    TRY(up32(&ctx->prec_out32, f32.prec_out));
    TRY(up64(&ctx->proj_b, f64.proj_b));
    TRY(up64(&ctx->proj_bt, f64.proj_bt));
    TRY(up64(&ctx->proj_kab, f64.proj_kab));
    {
      // multiplier block of every element facet: interior facets keep their
      // id, wall facets follow in element order
      std::vector<int32_t> mf(ctx->mesh.fid);
      int64_t w = 0;
      for (auto& v : mf)
        if (v < 0) v = (int32_t)(ctx->mesh.F + w++);
      TRY(upload(ctx, &ctx->mfid, mf));
    }
    ctx->vol_dV64 = a.vol_dV;
    // workspaces
    const int64_t E = n_elems, n = ctx->n_dof;
    TRY(dev_alloc(ctx, &ctx->m64, (size_t)E * s.nm));
    TRY(dev_alloc(ctx, &ctx->m32, (size_t)E * s.nm));
    TRY(dev_alloc(ctx, &ctx->mu64, (size_t)E * s.nm));
    TRY(dev_alloc(ctx, &ctx->mu32, (size_t)E * s.nm));
    // element slots (E * nfl) or the mass kernels' facet-side rows (2 F nf
    // <= E nfl) followed by their trash slots
    TRY(dev_alloc(ctx, &ctx->slot, (size_t)E * s.nfl + 128));
    ctx->npart = std::max<int64_t>(std::max<int64_t>(2 * NPART, ctx->bat.nb), (E + 15) / 16);
    TRY(dev_alloc(ctx, &ctx->part, (size_t)ctx->npart));
    TRY(dev_alloc(ctx, &ctx->part2, (size_t)(2 * NPART)));
    TRY(dev_alloc(ctx, &ctx->r, (size_t)n));
    TRY(dev_alloc(ctx, &ctx->z, (size_t)n));
    {
      // direction history: up to 64 vectors within 32 GB (an eighth of the
      // GPU's memory), at least 4 (HOPU_TEST_RING=h sets h, for tests of the
      // ring's wrap-around).  A solve checks convergence at most every
      // nph - 1 iterations, and each check adds the directions since the
      // last one to x in one pass (x read and written once per chunk).
      const int64_t fit = (int64_t)(32.0e9 / (8.0 * (double)std::max<int64_t>(n, 1)));
      ctx->nph = (int)std::max<int64_t>(4, std::min<int64_t>(64, fit));
      const char* ring = std::getenv("HOPU_TEST_RING");
      if (ring && std::atoi(ring) >= 2 && std::atoi(ring) <= 64) ctx->nph = std::atoi(ring);
      TRY(dev_alloc(ctx, &ctx->phist, (size_t)ctx->nph * (size_t)n));
      TRY(dev_alloc(ctx, &ctx->ahist, (size_t)ctx->nph));
    }
    TRY(dev_alloc(ctx, &ctx->q, (size_t)n));
    TRY(dev_alloc(ctx, &ctx->stage, (size_t)n));
    TRY(dev_alloc(ctx, &ctx->w, (size_t)n));
    TRY(dev_alloc(ctx, &ctx->rc, (size_t)n));
    for (int i = 0; i < 3; ++i) TRY(dev_alloc(ctx, &ctx->wh[i], (size_t)n));
    TRY(dev_alloc(ctx, &ctx->sc, SC_N));
    TRY(dev_alloc(ctx, &ctx->own_lfac, (size_t)ctx->mesh.F));
    TRY(dev_alloc(ctx, &ctx->eta_nd, (size_t)(2 * ctx->mesh.F)));
    TRY(dev_alloc(ctx, &ctx->flag, 4));
    TRY(dev_alloc(ctx, &ctx->nbad, 1));
    void* hp = nullptr;
    if (hipHostMalloc(&hp, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) { st = HOPU_ENOMEM; ctx->err = "hipHostMalloc failed"; goto fail_create; }
    ctx->hflag = (int*)hp;
    // this device's evaluation scratch (set up once per device, here, with
    // the context's device current)
    if ((st = scratch_address(&ctx->eval_scratch, ctx->err)) != HOPU_OK) goto fail_create;
    if (hipMemsetAsync(ctx->w, 0, n * sizeof(double), ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->slot, 0, (size_t)E * s.nfl * sizeof(double), ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
      st = HOPU_EHIP;
      ctx->err = "initial device copies failed";
      goto fail_create;
    }
  }
  *out = ctx;
  return HOPU_OK;
fail_create:
  g_create_err = ctx->err;
  hopu_destroy(ctx);
  return st;
#undef TRY
}

extern "C" void hopu_destroy(hopu_ctx ctx) {
  if (!ctx) return;
  if (!ctx->allocs.empty()) {
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
  }
  for (hipEvent_t ev : ctx->events) (void)hipEventDestroy(ev);
  for (void* p : ctx->allocs) (void)hipFree(p);
  if (ctx->hflag) (void)hipHostFree(ctx->hflag);
  delete ctx;
}

extern "C" const char* hopu_last_error(hopu_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

extern "C" hopu_status hopu_sizes(hopu_ctx ctx, int64_t* n_dof, int64_t* n_facets, int64_t* n_wall_facets, int* n_loc,
                                  int* n_facet_dof, int* n_interior_dof) {
  if (!ctx) return HOPU_EINVAL;
  if (n_dof) *n_dof = ctx->n_dof;
  if (n_facets) *n_facets = ctx->mesh.F;
  if (n_wall_facets) *n_wall_facets = ctx->mesh.W;
  if (n_loc) *n_loc = ctx->sz.n;
  if (n_facet_dof) *n_facet_dof = ctx->sz.nf;
  if (n_interior_dof) *n_interior_dof = ctx->sz.nint;
  return HOPU_OK;
}

extern "C" hopu_status hopu_set_upwind(hopu_ctx ctx, int l_global, const int8_t* l_per_facet_dev) {
  if (!ctx) return HOPU_EINVAL;
  if (l_global < -1 || l_global > ctx->k) return fail(ctx, HOPU_EINVAL, "l must be in -1..k");
  ctx->adapt_every = 0;  // an explicit choice replaces the adaptive order
  ctx->lglob = l_global;
  ctx->lfac = l_per_facet_dev;
  refresh_dm(ctx);
  return HOPU_OK;
}

extern "C" hopu_status hopu_set_solver(hopu_ctx ctx, double rtol, int max_it, int check_every) {
  if (!ctx) return HOPU_EINVAL;
  if (!(rtol > 0) || max_it < 1 || check_every < 1) return fail(ctx, HOPU_EINVAL, "rtol > 0, max_it >= 1, check_every >= 1");
  ctx->rtol = rtol;
  ctx->max_it = max_it;
  ctx->check_every = check_every;
  return HOPU_OK;
}

// ------------------------------------------------------------------ internals
static hopu_status do_modal(hopu_ctx ctx, const double* u, hopu_precision prec, bool second = false) {
  double* d64 = second ? ctx->mu64 : ctx->m64;
  float* d32 = second ? ctx->mu32 : ctx->m32;
  // the persistent mass kernel's gather reads a facet's rows in 16-byte pairs
  if (reinterpret_cast<uintptr_t>(u) % 16 != 0) {
    vec_copy(ctx->stream, ctx->stage, u, ctx->n_dof);
    u = ctx->stage;
  }
  prof_begin(ctx, PROF_MODAL);
  DISPATCH(ctx->dim, ctx->k, {
    // FP64 transform in every form; FP32 store for the reduced ones
    const bool f32 = prec != HOPU_FP64;
    void* dst = f32 ? static_cast<void*>(d32) : static_cast<void*>(d64);
    if (!launch_modal_mass<D, KK>(ctx->stream, u, dst, f32, ctx->slot, ctx->dm, ctx->mass_in)) {
      if (f32) launch_modal<float, D, KK>(ctx->stream, u, d32, ctx->dm, ctx->tb64.modal);
      else launch_modal<double, D, KK>(ctx->stream, u, d64, ctx->dm, ctx->tb64.modal);
    }
  });
  prof_end(ctx);
  return HOPU_OK;
}

static hopu_status do_apply(hopu_ctx ctx, const double* u, double* r, int terms, hopu_precision prec,
                            double* diss_part, double* eta_nd = nullptr) {
  hopu_status st = do_modal(ctx, u, prec);
  if (st) return st;
  prof_begin(ctx, PROF_ELEM);
  DISPATCH(ctx->dim, ctx->k, {
    if (prec == HOPU_FP64) launch_elem<double, D, KK>(ctx->stream, ctx->m64, r, ctx->slot, ctx->dm, ctx->tb64, terms, diss_part, eta_nd);
    else if (prec == HOPU_BF16X2) launch_elem_bf<2, D, KK>(ctx->stream, ctx->m32, r, ctx->slot, ctx->dm, ctx->tbb2, terms, diss_part);
    else if (prec == HOPU_BF16X3) launch_elem_bf<3, D, KK>(ctx->stream, ctx->m32, r, ctx->slot, ctx->dm, ctx->tbb3, terms, diss_part);
    else launch_elem<float, D, KK>(ctx->stream, ctx->m32, r, ctx->slot, ctx->dm, ctx->tb32, terms, diss_part, eta_nd);
  });
  prof_end(ctx);
  DISPATCH(ctx->dim, ctx->k, { launch_assemble<D, KK>(ctx->stream, r, ctx->slot, ctx->dm, nullptr); });
  return HOPU_OK;
}

// y = M x (mode 0) or the preconditioner (mode 1), unassembled: interior rows
// of y plus the facet-side contributions in ctx->slot (the facet rows of y
// are left untouched).  With `dot`, the per-block partials of x . y go to
// ctx->part; returns their number.
static int mass_raw(hopu_ctx ctx, int mode, const double* x, double* y, const int* flag, bool in_loop, bool dot,
                    bool prec32 = false) {
  int np = 0;
  // the 3D kernels read a facet's rows in 16-byte pairs
  if (reinterpret_cast<uintptr_t>(x) % 16 != 0) {
    vec_copy(ctx->stream, ctx->stage, x, ctx->n_dof);
    x = ctx->stage;
  }
  prof_begin(ctx, in_loop ? (mode == 0 ? PROF_MASS : PROF_PREC) : PROF_PLAIN);
  DISPATCH(ctx->dim, ctx->k, {
    np = launch_mass<D, KK>(ctx->stream, mode, x, y, ctx->slot, ctx->dm, mode == 0 ? ctx->mass_in : ctx->prec_in,
                            mode == 0 ? ctx->mass_out : ctx->prec_out, flag, dot ? ctx->part : nullptr,
                            prec32 ? ctx->prec_in32 : nullptr, prec32 ? ctx->prec_out32 : nullptr);
  });
  prof_end(ctx);
  return np;
}

// y = M x (mode 0) or the preconditioner (mode 1), assembled
static void do_mass(hopu_ctx ctx, int mode, const double* x, double* y, const int* flag) {
  mass_raw(ctx, mode, x, y, flag, false, false);
  launch_fs_assemble(ctx->stream, y, ctx->slot, ctx->mesh.F * ctx->sz.nf, flag);
}

static hopu_status check_prec(hopu_ctx ctx, hopu_precision prec) {
  if ((int)prec < (int)HOPU_FP64 || (int)prec > (int)HOPU_BF16X3) return fail(ctx, HOPU_EINVAL, "unknown precision");
  return HOPU_OK;
}

extern "C" hopu_status hopu_convection_apply(hopu_ctx ctx, const double* u, double* r, int terms, hopu_precision prec) {
  RocRange range("hopu_convection_apply");
  if (!ctx) return HOPU_EINVAL;
  if (!u || !r) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (terms < 0 || terms > 7) return fail(ctx, HOPU_EINVAL, "terms must be a HOPU_TERM_* mask");
  if (check_prec(ctx, prec)) return HOPU_EINVAL;
  refresh_dm(ctx);
  hopu_status st = do_apply(ctx, u, r, terms, prec, nullptr);
  if (st) return st;
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

extern "C" hopu_status hopu_mass_apply(hopu_ctx ctx, const double* u, double* y) {
  if (!ctx) return HOPU_EINVAL;
  if (!u || !y) return fail(ctx, HOPU_EINVAL, "NULL vector");
  do_mass(ctx, 0, u, y, nullptr);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

// PCG on M with R blockdiag(M_T)^-1 R^t; x holds the initial guess.
// prec32: the preconditioner's contractions in FP32 MFMA (the mixed-precision
// substeps); M, the vectors and the inner products stay FP64, so the solution
// meets the same tolerance
static hopu_status pcg(hopu_ctx ctx, const double* b, double* x, double rtol, int max_it, int* iters,
                       bool prec32 = false) {
  const int64_t n = ctx->n_dof;
  hipStream_t s = ctx->stream;
  int* fl = ctx->flag;
  const int64_t nfl = ctx->mesh.F * ctx->sz.nf;
  HCHECK(hipMemsetAsync(fl, 0, 4 * sizeof(int), s));
  // tolerance from b.Pb
  int np = mass_raw(ctx, 1, b, ctx->z, nullptr, false, true, prec32);
  vec_scalar(s, ctx->part, np, ctx->sc, fl, OP_SET_TOL, rtol, nullptr);
  // r = b - M x; z = P r (assembled straight into p); p = z
  mass_raw(ctx, 0, x, ctx->q, nullptr, false, false);
  vec_sub_fs(s, ctx->r, b, ctx->q, ctx->slot, nfl, n);
  const int H = ctx->nph;
  auto pdir = [&](int64_t i) { return ctx->phist + (i % H) * n; };
  np = mass_raw(ctx, 1, ctx->r, pdir(0), nullptr, false, true, prec32);
  launch_fs_assemble(s, pdir(0), ctx->slot, nfl, nullptr);
  vec_scalar(s, ctx->part, np, ctx->sc, fl, OP_SET_RZ, 0.0, nullptr);
  int it = 0;
  int flushed = 0;  // x holds x_0 + sum_{i < flushed} alpha_i p_i
  bool conv = false;
  // the first chunk runs one iteration more than the previous solve needed
  // (warm-started solves converge in similar counts, so most solves end in
  // it with a single host check; iterations queued past convergence return
  // at once), then check_every.
  // q = M p and z = P r stay unassembled: their facet rows are summed from
  // the facet-side buffer by the update that reads them, and p . q, r . z
  // come from the mass kernels' element-local partials.  p_i lives in ring
  // slot i % H; a chunk never overwrites a direction not yet added to x.
  std::vector<size_t> prof_idx;  // profile pairs of each launched iteration
  while (it < max_it) {
    const int want = (it == 0 && ctx->last_its > 0) ? ctx->last_its + 1 : ctx->check_every;
    const int chunk = std::min(std::min(want, max_it - it), H - 1 - (it - flushed));
    for (int c = 0; c < chunk; ++c) {
      const int64_t i = it + c;
      prof_idx.push_back(ctx->ev_used);
      np = mass_raw(ctx, 0, pdir(i), ctx->q, fl, true, true);
      // alpha (recorded for the solution update); r -= alpha q
      vec_rupdate(s, ctx->r, ctx->q, ctx->slot, nfl, n, ctx->sc, fl, ctx->part, np, nullptr, ctx->ahist + i % H);
      np = mass_raw(ctx, 1, ctx->r, ctx->z, fl, true, true, prec32);
      // beta, test; p_{i+1} = z + beta p_i
      vec_xpay(s, nullptr, pdir(i), pdir(i + 1), ctx->z, ctx->slot, nfl, n, ctx->sc, fl, ctx->part, np);
    }
    it += chunk;
    HCHECK(hipMemcpyAsync(ctx->hflag, fl, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    // every iteration counted in flag[1] has its alpha and direction (the
    // one that converged included); those queued after it did nothing
    const int ran = ctx->hflag[1];
    if (ran > flushed) vec_xflush(s, x, ctx->phist, ctx->ahist, n, H, flushed, ran - flushed);
    flushed = ran;
    if (ctx->hflag[0]) { conv = true; break; }
  }
  const int done = ctx->hflag[1];
  HCHECK(hipGetLastError());
  // launches queued after convergence returned at once: keep them out of the
  // per-kernel timing (the timed launches from iteration `done` on)
  if (ctx->prof && (size_t)std::max(done, 0) < prof_idx.size())
    for (size_t e2 = prof_idx[(size_t)std::max(done, 0)]; e2 < ctx->ev_used; ++e2) ctx->ev_kind[e2] = -1;
  ctx->last_its = done;
  if (iters) *iters = done;
  if (!conv) {
    ctx->err = "PCG did not reach rtol within max_it iterations";
    return HOPU_ENOCONV;
  }
  return HOPU_OK;
}

// Projection step (paper section 2.3, eq. (MCS_step2); u_new = u* - u~):
// CG on the condensed multiplier system S_p p^ = g (unpreconditioned), then
// the element-wise recovery of u~.
extern "C" hopu_status hopu_project(hopu_ctx ctx, const double* ustar, double* unew, double rtol, int max_it,
                                    int* iters) {
  RocRange range("hopu_project");
  if (!ctx) return HOPU_EINVAL;
  if (!ustar || !unew) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (ustar == unew) return fail(ctx, HOPU_EINVAL, "u* and u_new must be different vectors");
  if (!(rtol > 0.0) || max_it < 1) return fail(ctx, HOPU_EINVAL, "rtol must be > 0 and max_it >= 1");
  hipStream_t s = ctx->stream;
  const int nQ = ctx->sz.dim == 2 ? ctx->k * (ctx->k + 1) / 2 : ctx->k * (ctx->k + 1) * (ctx->k + 2) / 6;
  const int64_t FW = ctx->mesh.F + ctx->mesh.W;
  const int64_t nh = FW * ctx->sz.nf;
  ProjDev pj{ctx->mfid, FW, ctx->mass_in, ctx->prec_in, ctx->prec_out, ctx->proj_b, ctx->proj_bt, nullptr};
  if (!ctx->proj_ready) {
    hopu_status st;
    // direction ring: one chunk of 16 iterations and the next direction,
    // within 8 GB (at least 4)
    const int64_t fit = (int64_t)(8.0e9 / (8.0 * (double)std::max<int64_t>(nh, 1)));
    ctx->npph = (int)std::max<int64_t>(4, std::min<int64_t>(17, fit));
    if ((st = dev_alloc(ctx, &ctx->ainv, (size_t)ctx->mesh.E * nQ * nQ)) ||
        (st = dev_alloc(ctx, &ctx->ph, (size_t)nh)) || (st = dev_alloc(ctx, &ctx->pr, (size_t)nh)) ||
        (st = dev_alloc(ctx, &ctx->pfs, (size_t)2 * nh)) ||
        (st = dev_alloc(ctx, &ctx->pph, (size_t)ctx->npph * (size_t)nh)) ||
        (st = dev_alloc(ctx, &ctx->paht, (size_t)ctx->npph)))
      return st;
    // wall facets have one side: their second contribution stays zero
    HCHECK(hipMemsetAsync(ctx->pfs, 0, (size_t)2 * nh * sizeof(double), s));
    DISPATCH(ctx->dim, ctx->k, { launch_proj_ainv<D, KK>(s, ctx->dm, ctx->proj_kab, ctx->ainv); });
    HCHECK(hipGetLastError());
    ctx->proj_ready = true;
  }
  pj.ainv = ctx->ainv;
  int* fl = ctx->flag;
  HCHECK(hipMemsetAsync(fl, 0, 4 * sizeof(int), s));
  HCHECK(hipMemsetAsync(ctx->ph, 0, (size_t)nh * sizeof(double), s));
  // r = g, p = r
  DISPATCH(ctx->dim, ctx->k, { launch_proj<D, KK>(s, 1, nullptr, ustar, ctx->pfs, ctx->dm, pj, nullptr); });
  launch_fs_assemble(s, ctx->pr, ctx->pfs, nh, nullptr);
  const int H = ctx->npph;
  auto pdir = [&](int64_t i) { return ctx->pph + (i % H) * nh; };
  vec_copy(s, pdir(0), ctx->pr, nh);
  // ||r|| <= rtol (||g||^2 + ||u*_F||^2)^1/2: the facet block of u* (same
  // units as g) keeps the criterion meaningful when u* is (nearly)
  // divergence-free and g is rounding noise
  vec_dot(s, ctx->pr, ctx->pr, nh, ctx->part, nullptr);
  vec_dot(s, ustar, ustar, ctx->mesh.F * ctx->sz.nf, ctx->part + NPART, nullptr);
  vec_scalar(s, ctx->part, 2 * NPART, ctx->sc, fl, OP_SET_TOL, rtol, nullptr);
  vec_dot(s, ctx->pr, ctx->pr, nh, ctx->part, nullptr);
  vec_scalar(s, ctx->part, NPART, ctx->sc, fl, OP_SET_RZ, 0.0, nullptr);
  int it = 0;
  int flushed = 0;  // ph holds sum_{i < flushed} alpha_i p_i
  bool conv = false;
  // the solution update is made from the ring at each host check, as in
  // the PCG (one pass over the directions instead of an x read and write
  // per iteration)
  while (it < max_it) {
    const int chunk = std::min(std::min(16, max_it - it), H - 1 - (it - flushed));
    for (int c = 0; c < chunk; ++c) {
      const int64_t i = it + c;
      int np = 0;
      DISPATCH(ctx->dim, ctx->k, { np = launch_proj<D, KK>(s, 0, pdir(i), nullptr, ctx->pfs, ctx->dm, pj, ctx->part, fl); });
      // alpha (recorded); r -= alpha S_p p; partials of r.r into part2
      const int nr = vec_rupdate(s, ctx->pr, ctx->pr, ctx->pfs, nh, nh, ctx->sc, fl, ctx->part, np, ctx->part2,
                                 ctx->paht + i % H);
      // beta, test; p_{i+1} = r + beta p_i
      vec_xpay(s, nullptr, pdir(i), pdir(i + 1), ctx->pr, ctx->pfs, 0, nh, ctx->sc, fl, ctx->part2, nr);
    }
    it += chunk;
    HCHECK(hipMemcpyAsync(ctx->hflag, fl, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HCHECK(hipStreamSynchronize(s));
    const int ran = ctx->hflag[1];
    if (ran > flushed) vec_xflush(s, ctx->ph, ctx->pph, ctx->paht, nh, H, flushed, ran - flushed);
    flushed = ran;
    if (ctx->hflag[0]) { conv = true; break; }
  }
  const int done = ctx->hflag[1];
  // u_new = u* - u~
  DISPATCH(ctx->dim, ctx->k, { launch_proj<D, KK>(s, 2, ctx->ph, ustar, unew, ctx->dm, pj, nullptr); });
  HCHECK(hipGetLastError());
  if (iters) *iters = done;
  if (!conv) {
    ctx->err = "projection CG did not reach rtol within max_it iterations";
    return HOPU_ENOCONV;
  }
  return HOPU_OK;
}

// Measurement: the FP64 MFMA rate this GPU sustains with blocks_per_cu
// blocks of four waves per CU (waves per SIMD = blocks_per_cu).
extern "C" hopu_status hopu_mfma_f64_rate(int blocks_per_cu, double* tflops) {
  if (blocks_per_cu < 1 || blocks_per_cu > 8 || !tflops) return HOPU_EINVAL;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return HOPU_EHIP;
  const int blocks = cus * blocks_per_cu, iters = 4000;
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hopu_status st = HOPU_OK;
  float ms = 0.f;
  if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(double)) != hipSuccess) return HOPU_ENOMEM;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { st = HOPU_EHIP; goto done; }
  launch_mfma_f64_rate(nullptr, out, blocks, iters);  // warm-up (clocks)
  if (hipEventRecord(e0, nullptr) != hipSuccess) { st = HOPU_EHIP; goto done; }
  launch_mfma_f64_rate(nullptr, out, blocks, iters);
  if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = HOPU_EHIP; goto done; }
  *tflops = (double)blocks * 4 * iters * 8 * 2048.0 / (ms * 1e-3) / 1e12;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return st;
}

extern "C" hopu_status hopu_mass_solve(hopu_ctx ctx, const double* r, double* w, double rtol, int max_it, int* iters) {
  RocRange range("hopu_mass_solve");
  if (!ctx) return HOPU_EINVAL;
  if (!r || !w) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (max_it < 1) return fail(ctx, HOPU_EINVAL, "max_it must be >= 1");
  return pcg(ctx, r, w, rtol > 0 ? rtol : ctx->rtol, max_it, iters);
}

static hopu_status diag_into(hopu_ctx ctx, const double* u, double* dst /*dev [3]*/, bool have_modal_and_diss,
                             int64_t ndiss) {
  // energy 1/2 u.Mu into dst[0] and ||div u||_L2 into dst[1], from the FP64
  // modal coefficients of u
  hipStream_t s = ctx->stream;
  if (!have_modal_and_diss) {
    do_modal(ctx, u, HOPU_FP64);
  }
  int64_t nw = 0;
  DISPATCH(ctx->dim, ctx->k, {
    launch_energy<D, KK>(s, ctx->m64, ctx->dm, ctx->part);
    vec_scalar(s, ctx->part, AUX_NPART, ctx->sc, ctx->flag, OP_STORE, 0.0, dst + 0);
    nw = launch_div<D, KK>(s, ctx->m64, ctx->dm, ctx->vol_dV64, ctx->tb64.wv, ctx->part);
    // ||div u||_L2: the square root of the summed squares, taken on the device
    vec_scalar(s, ctx->part, (int)nw, ctx->sc, ctx->flag, OP_STORE_SQRT, 0.0, dst + 1);
  });
  (void)ndiss;
  return HOPU_OK;
}

extern "C" hopu_status hopu_count_nonfinite(hopu_ctx ctx, const double* v, int64_t* count) {
  if (!ctx) return HOPU_EINVAL;
  if (!v || !count) return fail(ctx, HOPU_EINVAL, "NULL pointer");
  launch_count_nonfinite(ctx->stream, v, ctx->n_dof, ctx->nbad);
  unsigned long long h = 0;
  HCHECK(hipMemcpyAsync(&h, ctx->nbad, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  HCHECK(hipStreamSynchronize(ctx->stream));
  *count = (int64_t)h;
  return HOPU_OK;
}

extern "C" hopu_status hopu_energy(hopu_ctx ctx, const double* u, double* energy_dev) {
  if (!ctx) return HOPU_EINVAL;
  if (!u || !energy_dev) return fail(ctx, HOPU_EINVAL, "NULL pointer");
  hopu_status st = do_modal(ctx, u, HOPU_FP64);
  if (st) return st;
  DISPATCH(ctx->dim, ctx->k, {
    launch_energy<D, KK>(ctx->stream, ctx->m64, ctx->dm, ctx->part);
    vec_scalar(ctx->stream, ctx->part, AUX_NPART, ctx->sc, ctx->flag, OP_STORE, 0.0, energy_dev);
  });
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

extern "C" hopu_status hopu_diagnostics(hopu_ctx ctx, const double* u, double* energy, double* div_l2,
                                        double* dissipation) {
  if (!ctx) return HOPU_EINVAL;
  if (!u) return fail(ctx, HOPU_EINVAL, "NULL vector");
  refresh_dm(ctx);
  hipStream_t s = ctx->stream;
  double* const dd = ctx->z;  // three device scalars (z is free outside the PCG)
  // dissipation: run the element kernel with facet terms and collect partials
  hopu_status st = do_apply(ctx, u, ctx->rc, HOPU_TERM_UPWIND, HOPU_FP64, ctx->part);
  if (st) return st;
  vec_scalar(s, ctx->part, (int)ctx->bat.nb, ctx->sc, ctx->flag, OP_STORE, 0.0, dd + 2);
  diag_into(ctx, u, dd, true, 0);
  double h[3];
  HCHECK(hipMemcpyAsync(h, dd, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HCHECK(hipStreamSynchronize(s));
  if (energy) *energy = h[0];
  if (div_l2) *div_l2 = h[1];
  if (dissipation) *dissipation = h[2];
  return HOPU_OK;
}

// ------------------------------------------------------------------ adaptive order
// jump indicator of u with the facet orders in use (FP64 facet pass)
static hopu_status eta_pass(hopu_ctx ctx, const double* u) {
  refresh_dm(ctx);
  return do_apply(ctx, u, ctx->rc, HOPU_TERM_ALL, HOPU_FP64, nullptr, ctx->eta_nd);
}

extern "C" hopu_status hopu_jump_indicator(hopu_ctx ctx, const double* u, double* eta_dev) {
  if (!ctx) return HOPU_EINVAL;
  if (!u || !eta_dev) return fail(ctx, HOPU_EINVAL, "NULL vector");
  hopu_status st = eta_pass(ctx, u);
  if (st) return st;
  launch_adapt(ctx->stream, ctx->eta_nd, ctx->mesh.F, nullptr, ctx->k, nullptr, eta_dev);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

extern "C" hopu_status hopu_set_adaptive(hopu_ctx ctx, int every, int n_thresholds, const double* thresholds,
                                         int l_initial) {
  if (!ctx) return HOPU_EINVAL;
  if (every <= 0) {
    ctx->adapt_every = 0;
    ctx->lfac = nullptr;
    refresh_dm(ctx);
    return HOPU_OK;
  }
  if (n_thresholds != ctx->k + 1 || !thresholds) return fail(ctx, HOPU_EINVAL, "need k+1 thresholds eta_0..eta_k");
  for (int i = 0; i <= ctx->k; ++i) {
    const double lo = i ? thresholds[i - 1] : 0.0;
    if (!(thresholds[i] > lo) || !(thresholds[i] < 1.0))
      return fail(ctx, HOPU_EINVAL, "thresholds must satisfy 0 < eta_0 < ... < eta_k < 1");
  }
  if (l_initial < -1 || l_initial > ctx->k) return fail(ctx, HOPU_EINVAL, "l_initial must be in -1..k");
  for (int i = 0; i <= ctx->k; ++i) ctx->thr[i] = thresholds[i];
  ctx->adapt_every = every;
  HCHECK(hipMemsetAsync(ctx->own_lfac, (int)(uint8_t)(int8_t)l_initial, ctx->mesh.F, ctx->stream));
  ctx->lfac = ctx->own_lfac;
  refresh_dm(ctx);
  return HOPU_OK;
}

static hopu_status adapt_now(hopu_ctx ctx, const double* u) {
  hopu_status st = eta_pass(ctx, u);
  if (st) return st;
  launch_adapt(ctx->stream, ctx->eta_nd, ctx->mesh.F, ctx->thr, ctx->k, ctx->own_lfac, nullptr);
  return HOPU_OK;
}

extern "C" hopu_status hopu_get_facet_orders(hopu_ctx ctx, int8_t* l_dev) {
  if (!ctx) return HOPU_EINVAL;
  if (!l_dev) return fail(ctx, HOPU_EINVAL, "NULL output");
  if (ctx->adapt_every <= 0) return fail(ctx, HOPU_EINVAL, "adaptive order not enabled (hopu_set_adaptive)");
  if (ctx->mesh.F > 0)
    HCHECK(hipMemcpyAsync(l_dev, ctx->own_lfac, ctx->mesh.F, hipMemcpyDeviceToDevice, ctx->stream));
  return HOPU_OK;
}

extern "C" hopu_status hopu_adapt_upwind(hopu_ctx ctx, const double* u) {
  if (!ctx) return HOPU_EINVAL;
  if (!u) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (ctx->adapt_every <= 0) return fail(ctx, HOPU_EINVAL, "adaptive order not enabled (hopu_set_adaptive)");
  hopu_status st = adapt_now(ctx, u);
  if (st) return st;
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

extern "C" hopu_status hopu_substeps(hopu_ctx ctx, double* u, double dt, int n_steps, hopu_precision prec,
                                     double* diag_dev) {
  RocRange range("hopu_substeps");
  if (!ctx) return HOPU_EINVAL;
  if (!u) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (n_steps < 0) return fail(ctx, HOPU_EINVAL, "n_steps must be >= 0");
  if (!(std::isfinite(dt))) return fail(ctx, HOPU_EINVAL, "dt must be finite");
  if (check_prec(ctx, prec)) return HOPU_EINVAL;
  refresh_dm(ctx);
  hipStream_t s = ctx->stream;
  // PCG initial guess: polynomial extrapolation of the previous solutions
  // (w_{n-1}; 2w_{n-1} - w_{n-2}; 3w_{n-1} - 3w_{n-2} + w_{n-3}), from this
  // call's earlier substeps, or also the previous call's (hopu_set_warm_start)
  double* wh[3] = {ctx->wh[0], ctx->wh[1], ctx->wh[2]};
  int nh = ctx->carry_warm ? ctx->nwh : 0;
  ctx->nwh = 0;  // until this call has left its history consistent
  for (int st_i = 0; st_i <= n_steps; ++st_i) {
    const bool last = st_i == n_steps;
    if (diag_dev) {
      double* row = diag_dev + (int64_t)st_i * 5;
      // dissipation of the current state (FP64 facet pass), energy, divergence
      hopu_status st = do_apply(ctx, u, ctx->rc, HOPU_TERM_UPWIND, HOPU_FP64, ctx->part);
      if (st) return st;
      vec_scalar(s, ctx->part, (int)ctx->bat.nb, ctx->sc, ctx->flag, OP_STORE, 0.0, row + 2);
      double* tmp = ctx->z;
      diag_into(ctx, u, tmp, true, 0);
      HCHECK(hipMemcpyAsync(row, tmp, 2 * sizeof(double), hipMemcpyDeviceToDevice, s));
      if (st_i == 0) HCHECK(hipMemsetAsync(row + 3, 0, 2 * sizeof(double), s));
    }
    if (last) break;
    if (ctx->adapt_every > 0 && st_i % ctx->adapt_every == 0) {
      hopu_status sa = adapt_now(ctx, u);
      if (sa) return sa;
    }
    RocRange step_range("substep");
    hopu_status st = do_apply(ctx, u, ctx->rc, HOPU_TERM_ALL, prec, nullptr);
    if (st) return st;
    double* w = wh[2];
    if (nh == 0) HCHECK(hipMemsetAsync(w, 0, ctx->n_dof * sizeof(double), s));
    else if (nh == 1) HCHECK(hipMemcpyAsync(w, wh[0], ctx->n_dof * sizeof(double), hipMemcpyDeviceToDevice, s));
    else if (nh == 2) vec_comb3(s, w, wh[0], wh[1], 2.0, -1.0, 0.0, ctx->n_dof);
    else vec_comb3(s, w, wh[0], wh[1], 3.0, -3.0, 1.0, ctx->n_dof);
    int its = 0;
    st = pcg(ctx, ctx->rc, w, ctx->rtol, ctx->max_it, &its, prec != HOPU_FP64);
    if (st) return st;
    if (diag_dev) vec_copy_diag(s, diag_dev + (int64_t)(st_i + 1) * 5 + 3, ctx->sc, ctx->flag);
    vec_axpy(s, u, w, -dt, ctx->n_dof);
    wh[2] = wh[1];
    wh[1] = wh[0];
    wh[0] = w;
    nh = std::min(nh + 1, 3);
  }
  for (int i = 0; i < 3; ++i) ctx->wh[i] = wh[i];
  ctx->nwh = nh;
  HCHECK(hipGetLastError());
  HCHECK(hipStreamSynchronize(s));
  return HOPU_OK;
}

extern "C" hopu_status hopu_set_warm_start(hopu_ctx ctx, int carry) {
  if (!ctx) return HOPU_EINVAL;
  if (carry != 0 && carry != 1) return fail(ctx, HOPU_EINVAL, "carry must be 0 or 1");
  ctx->carry_warm = carry == 1;
  return HOPU_OK;
}

// ------------------------------------------------------------------ interpolation / eval
extern "C" hopu_status hopu_interp_points(hopu_ctx ctx, int n1d, double* pts_facet, double* pts_vol) {
  if (!ctx) return HOPU_EINVAL;
  if (n1d < 1 || n1d > 64) return fail(ctx, HOPU_EINVAL, "n1d must be in 1..64");
  std::vector<ld> sp, sw, vp, vw;
  simplex_rule(ctx->dim - 1, n1d, sp, sw);
  simplex_rule(ctx->dim, n1d, vp, vw);
  std::vector<double> s(sp.begin(), sp.end()), v(vp.begin(), vp.end());
  double *ds = nullptr, *dv = nullptr;
  HCHECK(hipMalloc(&ds, s.size() * 8));
  HCHECK(hipMalloc(&dv, v.size() * 8));
  HCHECK(hipMemcpyAsync(ds, s.data(), s.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  HCHECK(hipMemcpyAsync(dv, v.data(), v.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  launch_interp_points(ctx->stream, ctx->dim, (int)sw.size(), ds, (int)vw.size(), dv, ctx->xyz, ctx->dm, pts_facet,
                       pts_vol);
  HCHECK(hipStreamSynchronize(ctx->stream));
  (void)hipFree(ds);
  (void)hipFree(dv);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

extern "C" hopu_status hopu_interpolate(hopu_ctx ctx, int n1d, const double* vals_facet, const double* vals_vol,
                                        double* u) {
  if (!ctx) return HOPU_EINVAL;
  if (n1d < 1 || n1d > 64 || !u || (!vals_facet && ctx->mesh.F > 0) || (!vals_vol && ctx->sz.nint > 0))
    return fail(ctx, HOPU_EINVAL, "bad interpolation arguments");
  const int dim = ctx->dim, k = ctx->k;
  const Sizes& sz = ctx->sz;
  std::vector<ld> sp, sw, vp, vw;
  simplex_rule(dim - 1, n1d, sp, sw);
  simplex_rule(dim, n1d, vp, vw);
  std::vector<double> ws(sw.begin(), sw.end()), wv(vw.begin(), vw.end());
  std::vector<double> psi(sw.size() * sz.nf), qm(vw.size() * std::max(1, sz.nint) * dim, 0.0);
  std::vector<ld> tmp(std::max(sz.nf, std::max(1, sz.nint) * dim));
  for (size_t q = 0; q < sw.size(); ++q) {
    facet_psi(dim, k, &sp[q * (dim - 1)], tmp.data());
    for (int j = 0; j < sz.nf; ++j) psi[q * sz.nf + j] = (double)tmp[j];
  }
  if (sz.nint > 0)
    for (size_t q = 0; q < vw.size(); ++q) {
      interior_tests(dim, k, &vp[q * dim], tmp.data());
      for (int m = 0; m < sz.nint * dim; ++m) qm[q * sz.nint * dim + m] = (double)tmp[m];
    }
  double *dws, *dwv, *dpsi, *dqm;
  HCHECK(hipMalloc(&dws, ws.size() * 8));
  HCHECK(hipMalloc(&dwv, wv.size() * 8));
  HCHECK(hipMalloc(&dpsi, psi.size() * 8));
  HCHECK(hipMalloc(&dqm, qm.size() * 8));
  HCHECK(hipMemcpyAsync(dws, ws.data(), ws.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  HCHECK(hipMemcpyAsync(dwv, wv.data(), wv.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  HCHECK(hipMemcpyAsync(dpsi, psi.data(), psi.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  HCHECK(hipMemcpyAsync(dqm, qm.data(), qm.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  launch_interpolate(ctx->stream, dim, (int)ws.size(), sz.nf, vals_facet, dws, dpsi, (int)wv.size(), sz.nint,
                     vals_vol, dwv, dqm, ctx->dm, u);
  HCHECK(hipStreamSynchronize(ctx->stream));
  (void)hipFree(dws); (void)hipFree(dwv); (void)hipFree(dpsi); (void)hipFree(dqm);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

static constexpr int MAX_NP = 84;  // dim P^k, up to 3D k = 6

// The reference basis phi_j at n_pts points into phi [n_pts][n][dim] (host).
static void eval_tabulate(hopu_ctx ctx, int n_pts, const double* ref_pts, double* phi) {
  const int dim = ctx->dim, k = ctx->k;
  const Sizes& sz = ctx->sz;
  ld val[MAX_NP], grad[MAX_NP * 3];
  for (int p = 0; p < n_pts; ++p) {
    ld x[3];
    for (int a = 0; a < dim; ++a) x[a] = ref_pts[p * dim + a];
    dubiner(dim, k, x, val, grad);
    for (int j = 0; j < sz.n; ++j)
      for (int a = 0; a < dim; ++a) {
        ld s = 0;
        for (int al = 0; al < sz.nP; ++al) s += ctx->eval_db.Dinv[(a * sz.nP + al) * sz.n + j] * val[al];
        phi[((size_t)p * sz.n + j) * dim + a] = (double)s;
      }
  }
}

extern "C" hopu_status hopu_eval(hopu_ctx ctx, const double* u, int n_pts, const double* ref_pts, double* vals) {
  if (!ctx) return HOPU_EINVAL;
  if (!u || !vals || !ref_pts || n_pts < 1) return fail(ctx, HOPU_EINVAL, "bad eval arguments");
  const Sizes& sz = ctx->sz;
  std::vector<double> phi((size_t)n_pts * sz.n * ctx->dim);
  eval_tabulate(ctx, n_pts, ref_pts, phi.data());
  double* dphi;
  HCHECK(hipMalloc(&dphi, phi.size() * 8));
  HCHECK(hipMemcpyAsync(dphi, phi.data(), phi.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  launch_eval(ctx->stream, ctx->dim, sz.n, sz.nf, sz.nint, n_pts, u, dphi, ctx->dm, vals);
  HCHECK(hipStreamSynchronize(ctx->stream));
  (void)hipFree(dphi);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

// The same evaluation with the basis table in this device's `scratch`
// (through its looked-up address) and the host table in a per-thread
// static buffer: no allocation on the device or the host.  Every entry of
// the table that the kernel reads is written by this call first, so
// nothing needs clearing.
static thread_local double t_eval_host[EVAL_SCRATCH_DOUBLES];

extern "C" hopu_status hopu_eval_noalloc(hopu_ctx ctx, const double* u, int n_pts, const double* ref_pts,
                                         double* vals) {
  if (!ctx) return HOPU_EINVAL;
  if (!u || !vals || !ref_pts || n_pts < 1) return fail(ctx, HOPU_EINVAL, "bad eval arguments");
  const Sizes& sz = ctx->sz;
  const int64_t need = (int64_t)n_pts * sz.n * ctx->dim;
  if (need > EVAL_SCRATCH_DOUBLES)
    return fail(ctx, HOPU_EINVAL,
                "n_pts too large for the allocation-free evaluation: the table needs " + std::to_string(need) +
                    " doubles, the scratch holds " + std::to_string(EVAL_SCRATCH_DOUBLES) + " (at most " +
                    std::to_string(EVAL_SCRATCH_DOUBLES / (sz.n * ctx->dim)) + " points at this order)");
  if (!ctx->eval_scratch) return fail(ctx, HOPU_EHIP, "no evaluation scratch on this device");
  eval_tabulate(ctx, n_pts, ref_pts, t_eval_host);
  HCHECK(hipMemcpyAsync(ctx->eval_scratch, t_eval_host, (size_t)need * 8, hipMemcpyHostToDevice, ctx->stream));
  launch_eval(ctx->stream, ctx->dim, sz.n, sz.nf, sz.nint, n_pts, u, ctx->eval_scratch, ctx->dm, vals);
  HCHECK(hipStreamSynchronize(ctx->stream));
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

// ------------------------------------------------------------------ host-only inspection
extern "C" int64_t hopu_host_sizes(int dim, int k, int which) {
  if ((dim != 2 && dim != 3) || k < 1 || k > 6) return -1;
  Sizes s = make_sizes(dim, k);
  switch (which) {
    case 0: return s.n;
    case 1: return s.nf;
    case 2: return s.nint;
    case 3: return s.nP;
    case 4: return s.nqv;
    case 5: return s.nqf;
    default: return -1;
  }
}

extern "C" int64_t hopu_host_tables(int dim, int k, int which, double* out, int64_t cap) {
  if ((dim != 2 && dim != 3) || k < 1 || k > 6 || (!out && cap > 0)) return -1;
  if (which >= 20 && which <= 25) {  // the Stokes step's reference tables
    StokesTables st;
    std::string serr;
    if (!make_stokes_tables(dim, k, st, serr)) return -2;
    const std::vector<double>* sv[6] = {&st.Ea, &st.Gc, &st.MpG, &st.TV, &st.Phi, &st.Mref};
    const std::vector<double>& v = *sv[which - 20];
    const int64_t nwr = std::min<int64_t>(cap, (int64_t)v.size());
    if (out && nwr > 0) std::memcpy(out, v.data(), nwr * sizeof(double));
    return (int64_t)v.size();
  }
  RefTables t;
  std::string err;
  if (!make_ref_tables(dim, k, t, err)) return -2;
  const std::vector<double>* v = nullptr;
  FragTables f32;
  BfTables bf;
  std::vector<double> bits;
  if (which >= 8 && which <= 16) {
    make_frag_tables(t, ROWMAP_F32, f32);
    if (which == 9 || which == 10 || which == 12 || which == 15 || which == 16) {
      make_bf16_tables(f32, t.sz, which == 9 ? 2 : 3, bf);
      const std::vector<uint16_t>& b =
          which == 12 ? bf.fac_Tr : which == 15 ? bf.vol_dV : which == 16 ? bf.vol_VT : bf.vol_dVT;
      bits.assign(b.begin(), b.end());
    }
  }
  switch (which) {
    case 0: v = &t.xv; break;
    case 1: v = &t.wv; break;
    case 2: v = &t.V; break;
    case 3: v = &t.sf; break;
    case 4: v = &t.wf; break;
    case 5: v = &t.Psi; break;
    case 6: v = &t.D; break;
    case 7: v = &t.Dinv; break;
    case 8: v = &f32.vol_dVT; break;
    case 11: v = &f32.fac_Tr; break;
    case 13: v = &f32.vol_dV; break;
    case 14: v = &f32.vol_VT; break;
    case 9:
    case 10:
    case 12:
    case 15:
    case 16: v = &bits; break;
    default: return -1;
  }
  int64_t nwr = std::min<int64_t>(cap, (int64_t)v->size());
  if (out && nwr > 0) std::memcpy(out, v->data(), nwr * sizeof(double));
  return (int64_t)v->size();
}

extern "C" int64_t hopu_host_mesh(int dim, int64_t n_elems, const int64_t* elem_vid, const double* elem_xyz, int which,
                                  void* out, int64_t cap) {
  if ((dim != 2 && dim != 3) || n_elems <= 0 || !elem_vid || !elem_xyz) return -1;
  MeshData m;
  std::string err;
  if (!build_mesh(dim, n_elems, elem_vid, elem_xyz, m, err)) return -2;
  auto put_i32 = [&](const std::vector<int32_t>& v) {
    if (out) std::memcpy(out, v.data(), std::min<int64_t>(cap, v.size()) * 4);
    return (int64_t)v.size();
  };
  switch (which) {
    case 0: return put_i32(m.fid);
    case 1: return put_i32(m.nbr);
    case 2: return put_i32(std::vector<int32_t>(m.nbr_face.begin(), m.nbr_face.end()));
    case 3:
      if (out) std::memcpy(out, m.geo.data(), std::min<int64_t>(cap, m.geo.size()) * 8);
      return (int64_t)m.geo.size();
    case 4: return put_i32(m.facet_elem);
    case 5: {
      Batches b;
      make_batches(m, b);
      return put_i32(b.elem);
    }
    case 6: {  // the Stokes step's per-element frames [E][64]
      std::vector<double> sg;
      make_stokes_geometry(dim, m.E, m.xyz, m.geo, m.fid, sg);
      if (out) std::memcpy(out, sg.data(), std::min<int64_t>(cap, sg.size()) * 8);
      return (int64_t)sg.size();
    }
    default: return -1;
  }
}

// ------------------------------------------------------------------ adjoint
static hopu_status do_vjp(hopu_ctx ctx, const double* u, const double* mu, double* out, hopu_precision prec) {
  do_modal(ctx, u, prec, false);
  do_modal(ctx, mu, prec, true);
  prof_begin(ctx, PROF_VJP);
  DISPATCH(ctx->dim, ctx->k, {
    if (prec == HOPU_FP64)
      launch_vjp<double, D, KK>(ctx->stream, ctx->m64, ctx->mu64, out, ctx->slot, ctx->dm, ctx->tb64, u, ctx->psi_n64);
    else if (prec == HOPU_BF16X2)
      launch_vjp_bf<2, D, KK>(ctx->stream, ctx->m32, ctx->mu32, out, ctx->slot, ctx->dm, ctx->tbb2, u, ctx->psi_n32);
    else if (prec == HOPU_BF16X3)
      launch_vjp_bf<3, D, KK>(ctx->stream, ctx->m32, ctx->mu32, out, ctx->slot, ctx->dm, ctx->tbb3, u, ctx->psi_n32);
    else
      launch_vjp<float, D, KK>(ctx->stream, ctx->m32, ctx->mu32, out, ctx->slot, ctx->dm, ctx->tb32, u, ctx->psi_n32);
  });
  prof_end(ctx);
  DISPATCH(ctx->dim, ctx->k, { launch_assemble<D, KK>(ctx->stream, out, ctx->slot, ctx->dm, nullptr); });
  return HOPU_OK;
}

extern "C" hopu_status hopu_convection_vjp(hopu_ctx ctx, const double* u, const double* mu, double* out,
                                           hopu_precision prec) {
  if (!ctx) return HOPU_EINVAL;
  if (!u || !mu || !out) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (check_prec(ctx, prec)) return HOPU_EINVAL;
  refresh_dm(ctx);
  do_vjp(ctx, u, mu, out, prec);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

static int64_t n_ckpt(int n_steps, int ck) { return (n_steps + ck - 1) / ck; }

extern "C" int64_t hopu_substeps_vjp_workspace(hopu_ctx ctx, int n_steps, int ckpt_every) {
  if (!ctx || n_steps < 0 || ckpt_every < 1) return HOPU_EINVAL;
  // checkpoints hold (state, PCG warm start); a segment buffer; 4 work vectors
  return (2 * n_ckpt(n_steps, ckpt_every) + ckpt_every + 4) * ctx->n_dof * (int64_t)sizeof(double);
}

// one explicit substep u <- u - dt M^-1 r(u), warm-starting PCG from w
static hopu_status substep(hopu_ctx ctx, double* u, double* w, double dt, hopu_precision prec) {
  hopu_status st = do_apply(ctx, u, ctx->rc, HOPU_TERM_ALL, prec, nullptr);
  if (st) return st;
  st = pcg(ctx, ctx->rc, w, ctx->rtol, ctx->max_it, nullptr, prec != HOPU_FP64);
  if (st) return st;
  vec_axpy(ctx->stream, u, w, -dt, ctx->n_dof);
  return HOPU_OK;
}

extern "C" hopu_status hopu_substeps_vjp(hopu_ctx ctx, const double* u0, double dt, int n_steps, int ckpt_every,
                                         const double* lam_N, double* lam_0, hopu_precision prec, void* ws,
                                         int64_t ws_bytes) {
  RocRange range("hopu_substeps_vjp");
  if (!ctx) return HOPU_EINVAL;
  if (!u0 || !lam_N || !lam_0 || !ws) return fail(ctx, HOPU_EINVAL, "NULL pointer");
  if (n_steps < 0 || ckpt_every < 1 || !std::isfinite(dt)) return fail(ctx, HOPU_EINVAL, "bad step arguments");
  if (check_prec(ctx, prec)) return HOPU_EINVAL;
  const int64_t need = hopu_substeps_vjp_workspace(ctx, n_steps, ckpt_every);
  if (ws_bytes < need) return fail(ctx, HOPU_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
  refresh_dm(ctx);
  hipStream_t s = ctx->stream;
  const int64_t n = ctx->n_dof;
  const size_t vb = n * sizeof(double);
  const int64_t nck = n_ckpt(n_steps, ckpt_every);
  double* base = (double*)ws;
  double* ck_u = base;                       // [nck][n]
  double* ck_w = ck_u + nck * n;             // [nck][n]
  double* seg = ck_w + nck * n;              // [ckpt_every][n]
  double* u = seg + (int64_t)ckpt_every * n; // work state
  double* lam = u + n;
  double* muw = lam + n;
  double* vo = muw + n;
  // forward: checkpoint (u, w) at every ckpt_every-th state
  HCHECK(hipMemcpyAsync(u, u0, vb, hipMemcpyDeviceToDevice, s));
  HCHECK(hipMemsetAsync(ctx->w, 0, vb, s));
  for (int st_i = 0; st_i < n_steps; ++st_i) {
    if (st_i % ckpt_every == 0) {
      const int64_t c = st_i / ckpt_every;
      HCHECK(hipMemcpyAsync(ck_u + c * n, u, vb, hipMemcpyDeviceToDevice, s));
      HCHECK(hipMemcpyAsync(ck_w + c * n, ctx->w, vb, hipMemcpyDeviceToDevice, s));
    }
    hopu_status st = substep(ctx, u, ctx->w, dt, prec);
    if (st) return st;
  }
  // reverse
  HCHECK(hipMemcpyAsync(lam, lam_N, vb, hipMemcpyDeviceToDevice, s));
  HCHECK(hipMemsetAsync(muw, 0, vb, s));
  for (int64_t c = nck - 1; c >= 0; --c) {
    const int s0 = (int)(c * ckpt_every), s1 = std::min(n_steps, s0 + ckpt_every);
    HCHECK(hipMemcpyAsync(seg, ck_u + c * n, vb, hipMemcpyDeviceToDevice, s));
    HCHECK(hipMemcpyAsync(u, ck_u + c * n, vb, hipMemcpyDeviceToDevice, s));
    HCHECK(hipMemcpyAsync(ctx->w, ck_w + c * n, vb, hipMemcpyDeviceToDevice, s));
    for (int st_i = s0; st_i < s1 - 1; ++st_i) {
      hopu_status st = substep(ctx, u, ctx->w, dt, prec);
      if (st) return st;
      HCHECK(hipMemcpyAsync(seg + (int64_t)(st_i - s0 + 1) * n, u, vb, hipMemcpyDeviceToDevice, s));
    }
    for (int st_i = s1 - 1; st_i >= s0; --st_i) {
      hopu_status st = pcg(ctx, lam, muw, ctx->rtol, ctx->max_it, nullptr);
      if (st) return st;
      do_vjp(ctx, seg + (int64_t)(st_i - s0) * n, muw, vo, prec);
      vec_axpy(s, lam, vo, -dt, n);
    }
  }
  HCHECK(hipMemcpyAsync(lam_0, lam, vb, hipMemcpyDeviceToDevice, s));
  HCHECK(hipGetLastError());
  HCHECK(hipStreamSynchronize(s));
  return HOPU_OK;
}

// ------------------------------------------------------------------ profiling
extern "C" hopu_status hopu_profile_enable(hopu_ctx ctx, int enable, int max_launches) {
  if (!ctx) return HOPU_EINVAL;
  if (enable < 0) return fail(ctx, HOPU_EINVAL, "enable must be >= 0");
  if (enable && max_launches < 1) return fail(ctx, HOPU_EINVAL, "max_launches must be >= 1");
  HCHECK(hipStreamSynchronize(ctx->stream));
  if (enable) {
    size_t need = 2 * (size_t)max_launches;
    while (ctx->events.size() < need) {
      hipEvent_t ev;
      HCHECK(hipEventCreate(&ev));
      ctx->events.push_back(ev);
    }
    ctx->ev_kind.assign(max_launches, -1);
  }
  ctx->ev_used = 0;
  ctx->prof = enable != 0;
  ctx->prof_stride = enable > 0 ? enable : 1;
  for (int64_t& c : ctx->prof_count) c = 0;
  ctx->prof_armed = false;
  return HOPU_OK;
}

extern "C" hopu_status hopu_profile_read(hopu_ctx ctx, int kind, int64_t* launches, double* total_ms) {
  if (!ctx || kind < 0 || kind >= PROF_N) return HOPU_EINVAL;
  HCHECK(hipStreamSynchronize(ctx->stream));
  int64_t n = 0;
  double tot = 0.0;
  for (size_t i = 0; i < ctx->ev_used; ++i) {
    if (ctx->ev_kind[i] != kind) continue;
    float ms = 0.f;
    HCHECK(hipEventElapsedTime(&ms, ctx->events[2 * i], ctx->events[2 * i + 1]));
    tot += ms;
    ++n;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = tot;
  return HOPU_OK;
}

// ---------------------------------------------------------------- Stokes
// Implicit Stokes step (paper section 2.2, spaces and forms; section 2.3,
// eq. (MCS_step1), static condensation, element-wise BDDC).
static bool stokes_supported(int dim, int k) { return (dim == 2 && k >= 1 && k <= 4) || (dim == 3 && k >= 1 && k <= 4); }

static int64_t stokes_n_uhat(hopu_ctx ctx) { return ctx->mesh.F * (ctx->dim - 1) * ctx->sz.nf; }

extern "C" hopu_status hopu_stokes_sizes(hopu_ctx ctx, int64_t* n_total, int64_t* n_uhat, int* n_elem_unknowns) {
  if (!ctx) return HOPU_EINVAL;
  const StokesDims sd = stokes_dims(ctx->dim, ctx->k);
  if (n_total) *n_total = ctx->n_dof + stokes_n_uhat(ctx);
  if (n_uhat) *n_uhat = stokes_n_uhat(ctx);
  if (n_elem_unknowns) *n_elem_unknowns = sd.nx;
  return HOPU_OK;
}

static hopu_status stokes_alloc(hopu_ctx ctx) {
  std::string err;
  StokesTables tb;
  if (!make_stokes_tables(ctx->dim, ctx->k, tb, err)) return fail(ctx, HOPU_EINVAL, err);
  const StokesDims& sd = tb.sd;
  if (sd.nx > 256 || sd.nx * sd.nx > sd.ng * sd.nsf || sd.nE * 9 > 256)
    return fail(ctx, HOPU_EUNSUPPORTED, "Stokes element sizes outside the kernels' limits");
  std::vector<double> sgeo;
  make_stokes_geometry(ctx->dim, ctx->mesh.E, ctx->mesh.xyz, ctx->mesh.geo, ctx->mesh.fid, sgeo);
  const int64_t E = ctx->mesh.E, nX = ctx->n_dof + stokes_n_uhat(ctx);
  // on a failure part-way, release what this call allocated, so that a later
  // set-up starts clean instead of allocating a second copy
  const size_t mark = ctx->allocs.size();
  auto undo = [&](hopu_status st) {
    (void)hipStreamSynchronize(ctx->stream);
    while (ctx->allocs.size() > mark) {
      (void)hipFree(ctx->allocs.back());
      ctx->allocs.pop_back();
    }
    return st;
  };
  hopu_status st;
  const double *Ea, *Gc, *MpG, *TV, *Phi, *Mref, *g;
  if ((st = upload(ctx, &Ea, tb.Ea)) || (st = upload(ctx, &Gc, tb.Gc)) || (st = upload(ctx, &MpG, tb.MpG)) ||
      (st = upload(ctx, &TV, tb.TV)) || (st = upload(ctx, &Phi, tb.Phi)) || (st = upload(ctx, &Mref, tb.Mref)) ||
      (st = upload(ctx, &g, sgeo)))
    return undo(st);
  const size_t nn = (size_t)E * stokes_packed_stride(sd.nx);
  if ((st = dev_alloc(ctx, &ctx->st_S, nn)) || (st = dev_alloc(ctx, &ctx->st_Sinv, nn)) ||
      (st = dev_alloc(ctx, &ctx->st_slot, (size_t)E * (ctx->dim + 1) * sd.nsd)) ||
      (st = dev_alloc(ctx, &ctx->st_r, (size_t)nX)) || (st = dev_alloc(ctx, &ctx->st_z, (size_t)nX)) ||
      (st = dev_alloc(ctx, &ctx->st_p, (size_t)nX)) || (st = dev_alloc(ctx, &ctx->st_q, (size_t)nX)) ||
      (st = dev_alloc(ctx, &ctx->st_b, (size_t)nX)) || (st = dev_alloc(ctx, &ctx->st_mu, (size_t)ctx->n_dof)) ||
      (st = dev_alloc(ctx, &ctx->st_conv, (size_t)ctx->n_dof)) || (st = dev_alloc(ctx, &ctx->st_part, 1024)) ||
      (st = dev_alloc(ctx, &ctx->st_bad, 4)))
    return undo(st);
  ctx->st_sd = sd;
  ctx->st_dv = StokesDev{Ea, Gc, MpG, TV, Phi, Mref, g, ctx->dm.fid, ctx->dm.facet_elem, ctx->dm.facet_local,
                         E, ctx->mesh.F, ctx->n_dof};
  ctx->st_alloc = true;
  return HOPU_OK;
}

extern "C" hopu_status hopu_stokes_setup(hopu_ctx ctx, double nu, double dt, int flags) {
  RocRange range("hopu_stokes_setup");
  if (!ctx) return HOPU_EINVAL;
  if (!(nu > 0.0) || !(dt > 0.0) || !std::isfinite(nu) || !std::isfinite(dt))
    return fail(ctx, HOPU_EINVAL, "nu and dt must be positive and finite");
  if (flags & ~HOPU_STOKES_FP32_PRECOND) return fail(ctx, HOPU_EINVAL, "unknown flags");
  if (!stokes_supported(ctx->dim, ctx->k))
    return fail(ctx, HOPU_EUNSUPPORTED, "the Stokes step is built for 2D and 3D k <= 4");
  hopu_status st;
  if (!ctx->st_alloc && (st = stokes_alloc(ctx))) return st;
  ctx->st_ready = false;
  hipStream_t s = ctx->stream;
  // the set-up's per-block scratch lives only for this call
  double* scratch = nullptr;
  const size_t nscr = stokes_setup_scratch(ctx->st_sd);
  if (const char* f = std::getenv("HOPU_TEST_FAIL_ALLOC"); f && std::atoi(f) == 1)
    return fail(ctx, HOPU_ENOMEM, "device allocation refused (HOPU_TEST_FAIL_ALLOC)");
  if (hipMalloc(&scratch, nscr * sizeof(double)) != hipSuccess)
    return fail(ctx, HOPU_ENOMEM, "hipMalloc of the Stokes set-up scratch failed");
  HCHECK(hipMemsetAsync(ctx->st_bad, 0, sizeof(int), s));
  const bool fp32 = (flags & HOPU_STOKES_FP32_PRECOND) != 0;
  launch_stokes_setup(s, ctx->st_sd, ctx->st_dv, nu, dt, ctx->st_S, ctx->st_Sinv,
                      fp32 ? reinterpret_cast<float*>(ctx->st_Sinv) : nullptr, scratch, ctx->st_bad);
  int bad = 0;
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipMemcpyAsync(&bad, ctx->st_bad, sizeof(int), hipMemcpyDeviceToHost, s);
  hipError_t e3 = hipStreamSynchronize(s);
  hipFree(scratch);
  HCHECK(e1);
  HCHECK(e2);
  HCHECK(e3);
  if (bad) return fail(ctx, HOPU_EINVAL, "an element matrix of the Stokes step is not positive definite");
  ctx->st_nu = nu;
  ctx->st_dt = dt;
  ctx->st_fp32 = fp32;
  ctx->st_ready = true;
  return HOPU_OK;
}

// the Stokes element product (S or C^-1), timed as its own kernel kind
static void stokes_gemv(hopu_ctx ctx, int inv, const double* x, double* y) {
  prof_begin(ctx, inv ? PROF_STOKES_C : PROF_STOKES_S);
  const float* a32 = (inv && ctx->st_fp32) ? reinterpret_cast<const float*>(ctx->st_Sinv) : nullptr;
  launch_stokes_gemv(ctx->stream, ctx->st_sd, ctx->st_dv, inv ? ctx->st_Sinv : ctx->st_S, a32, inv, x, y,
                     ctx->st_slot);
  prof_end(ctx);
}

static hopu_status stokes_check(hopu_ctx ctx) {
  if (!ctx->st_ready) return fail(ctx, HOPU_EINVAL, "hopu_stokes_setup has not been called");
  return HOPU_OK;
}

extern "C" hopu_status hopu_stokes_apply(hopu_ctx ctx, const double* x, double* y) {
  if (!ctx) return HOPU_EINVAL;
  if (!x || !y) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (x == y) return fail(ctx, HOPU_EINVAL, "x and y must be different vectors");
  if (hopu_status st = stokes_check(ctx)) return st;
  stokes_gemv(ctx, 0, x, y);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

extern "C" hopu_status hopu_stokes_precond(hopu_ctx ctx, const double* x, double* y) {
  if (!ctx) return HOPU_EINVAL;
  if (!x || !y) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (x == y) return fail(ctx, HOPU_EINVAL, "x and y must be different vectors");
  if (hopu_status st = stokes_check(ctx)) return st;
  stokes_gemv(ctx, 1, x, y);
  HCHECK(hipGetLastError());
  return HOPU_OK;
}

static hopu_status stokes_dot(hopu_ctx ctx, const double* a, const double* b, int64_t n, double* out) {
  const int np = launch_stokes_dot(ctx->stream, a, b, n, ctx->st_part);
  double h[1024];
  HCHECK(hipMemcpyAsync(h, ctx->st_part, np * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HCHECK(hipStreamSynchronize(ctx->stream));
  double v = 0.0;
  for (int i = 0; i < np; ++i) v += h[i];
  *out = v;
  return HOPU_OK;
}

extern "C" hopu_status hopu_stokes_step(hopu_ctx ctx, const double* un, int flags, double* x, double rtol,
                                        int max_it, int* iters) {
  RocRange range("hopu_stokes_step");
  if (!ctx) return HOPU_EINVAL;
  if (!un || !x) return fail(ctx, HOPU_EINVAL, "NULL vector");
  if (!(rtol > 0.0) || max_it < 1) return fail(ctx, HOPU_EINVAL, "rtol must be > 0 and max_it >= 1");
  if (flags & ~(HOPU_STOKES_CONVECTION | HOPU_STOKES_GUESS)) return fail(ctx, HOPU_EINVAL, "unknown flags");
  if (hopu_status st = stokes_check(ctx)) return st;
  hipStream_t s = ctx->stream;
  const int64_t nX = ctx->n_dof + stokes_n_uhat(ctx);
  const bool with_convection = (flags & HOPU_STOKES_CONVECTION) != 0;
  // b = [M u^n / dt - r(u^n); 0]
  do_mass(ctx, 0, un, ctx->st_mu, nullptr);
  if (with_convection) {
    refresh_dm(ctx);
    if (hopu_status st = do_apply(ctx, un, ctx->st_conv, 7, HOPU_FP64, nullptr)) return st;
  }
  launch_stokes_rhs(s, ctx->st_b, ctx->st_mu, with_convection ? ctx->st_conv : nullptr, ctx->st_dt, ctx->n_dof, nX);
  // PCG on S with C^-1 = R S_BDDC^-1 R^t from x = 0 or the caller's guess;
  // the stopping rule is relative to the C^-1 norm of b either way
  vec_copy(s, ctx->st_r, ctx->st_b, nX);
  stokes_gemv(ctx, 1, ctx->st_r, ctx->st_z);
  double bz = 0.0;
  if (hopu_status st = stokes_dot(ctx, ctx->st_r, ctx->st_z, nX, &bz)) return st;
  const double stop = rtol * std::sqrt(std::fabs(bz));
  double rz = bz;
  if (flags & HOPU_STOKES_GUESS) {
    // r = b - S x
    stokes_gemv(ctx, 0, x, ctx->st_q);
    launch_stokes_axpy(s, ctx->st_r, ctx->st_q, -1.0, nX);
    stokes_gemv(ctx, 1, ctx->st_r, ctx->st_z);
    if (hopu_status st = stokes_dot(ctx, ctx->st_r, ctx->st_z, nX, &rz)) return st;
  } else {
    HCHECK(hipMemsetAsync(x, 0, (size_t)nX * sizeof(double), s));
  }
  vec_copy(s, ctx->st_p, ctx->st_z, nX);
  int it = 0;
  bool conv = !(std::sqrt(std::fabs(rz)) > stop);
  while (!conv && it < max_it) {
    stokes_gemv(ctx, 0, ctx->st_p, ctx->st_q);
    double pq = 0.0;
    if (hopu_status st = stokes_dot(ctx, ctx->st_p, ctx->st_q, nX, &pq)) return st;
    const double alpha = rz / pq;
    launch_stokes_axpy(s, x, ctx->st_p, alpha, nX);
    launch_stokes_axpy(s, ctx->st_r, ctx->st_q, -alpha, nX);
    stokes_gemv(ctx, 1, ctx->st_r, ctx->st_z);
    double rz1 = 0.0;
    if (hopu_status st = stokes_dot(ctx, ctx->st_r, ctx->st_z, nX, &rz1)) return st;
    ++it;
    if (!std::isfinite(rz1)) break;
    if (std::sqrt(std::fabs(rz1)) <= stop) conv = true;
    launch_stokes_xpby(s, ctx->st_p, ctx->st_z, rz1 / rz, nX);
    rz = rz1;
  }
  HCHECK(hipGetLastError());
  HCHECK(hipStreamSynchronize(s));
  if (iters) *iters = it;
  if (!conv) return fail(ctx, HOPU_ENOCONV, "Stokes PCG did not reach rtol within max_it iterations");
  return HOPU_OK;
}
