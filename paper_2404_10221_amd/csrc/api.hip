// Host runtime of the C ABI declared in include/rsfde.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <dlfcn.h>

#include <algorithm>
#include <string>
#include <mutex>
#include <cmath>
#include <new>
#include <vector>

#include "dht.h"
#include "fields.h"
#include "krylov.h"
#include "pass.h"
#include "pass_sizes.h"
#include "rsfde.h"
#include "setup.h"

// ---------------------------------------------------------------------------
// Device scratch of rsfde_apply_prec_noalloc: a file-scope array (one copy per
// GPU, held until the process ends).  Host code never uses its name as an
// address: the device address is taken once per device with
// hipGetSymbolAddress (scratch_ptr) and passed to the kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[RSFDE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};
}  // namespace

// Device address of `scratch` on the current device (resolved on first use per
// device; later calls return the stored address).
static hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// per-length dispatch
// ---------------------------------------------------------------------------
#define RSFDE_DECL(L)                                                                        \
  template <>                                                                                \
  hipError_t launch_pass_L<double, L>(const PassArgs&, bool, int, hipStream_t, hipEvent_t,  \
                                      hipEvent_t);                                           \
  template <>                                                                                \
  hipError_t launch_pass_L<float, L>(const PassArgs&, bool, int, hipStream_t, hipEvent_t,   \
                                     hipEvent_t);                                            \
  template <>                                                                                \
  hipError_t launch_pass_batched_L<double, L>(const BLaunch&, int64_t, bool, int, hipStream_t, \
                                              hipEvent_t, hipEvent_t);                      \
  template <>                                                                                \
  hipError_t launch_pass_batched_L<float, L>(const BLaunch&, int64_t, bool, int, hipStream_t, \
                                             hipEvent_t, hipEvent_t);                       \
  template <>                                                                                \
  hipError_t launch_spectrum_L<L>(const double*, int, const cpx<double>*, double*, float*,  \
                                  double*, hipStream_t);                                     \
  template <>                                                                                \
  hipError_t launch_dht_L<L>(const DhtArgs&, hipStream_t);                          \
  template <>                                                                                \
  hipError_t launch_dht_batched_L<L>(const DBLaunch&, int64_t, bool, hipStream_t);           \
  template <>                                                                                \
  hipError_t launch_dht_tables_L<L>(int, const cpx<double>*, cpx<double>*, cpx<double>*,     \
                                    hipStream_t);
RSFDE_FOR_EACH_L(RSFDE_DECL)
#undef RSFDE_DECL

static bool supported_L(int L) {
  switch (L) {
#define RSFDE_CASE(LL) case LL:
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
    return true;
    default:
      return false;
  }
}

static hipError_t launch_pass(int L, bool fp32, const PassArgs& a, bool strided, hipStream_t s,
                              hipEvent_t ea = nullptr, hipEvent_t eb = nullptr) {
  switch (L) {
#define RSFDE_CASE(LL)                                                    \
  case LL:                                                                \
    return fp32 ? launch_pass_L<float, LL>(a, strided, a.var, s, ea, eb)  \
                : launch_pass_L<double, LL>(a, strided, a.var, s, ea, eb);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_pass_batched(int L, bool fp32, const BLaunch& bl, int64_t nblocks,
                                      bool strided, int var, hipStream_t s, hipEvent_t ea,
                                      hipEvent_t eb) {
  switch (L) {
#define RSFDE_CASE(LL)                                                                     \
  case LL:                                                                                 \
    return fp32 ? launch_pass_batched_L<float, LL>(bl, nblocks, strided, var, s, ea, eb)   \
                : launch_pass_batched_L<double, LL>(bl, nblocks, strided, var, s, ea, eb);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return hipErrorInvalidValue;
}

static void pass_shape_rt(int L, bool fp32, bool strided, int var, int* nt, int* ppt) {
  switch (L) {
#define RSFDE_CASE(LL)                                  \
  case LL:                                              \
    if (fp32) pass_shape<float, LL>(strided, var, nt, ppt); \
    else pass_shape<double, LL>(strided, var, nt, ppt);     \
    return;
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  *nt = 0;
  *ppt = 0;
}

static bool pass_plan_rt(int L, int var, int* code, int* radix, int* nstage) {
  switch (L) {
#define RSFDE_CASE(LL) \
  case LL:             \
    return pass_plan<LL>(var, code, radix, nstage);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return false;
}

static hipError_t launch_dht(int L, const DhtArgs& a, hipStream_t s) {
  switch (L) {
#define RSFDE_CASE(LL) \
  case LL:             \
    return launch_dht_L<LL>(a, s);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return hipErrorInvalidValue;
}

static hipError_t launch_dht_batched(int L, const DBLaunch& bl, int64_t nblocks, bool strided,
                                     hipStream_t s) {
  switch (L) {
#define RSFDE_CASE(LL) \
  case LL:             \
    return launch_dht_batched_L<LL>(bl, nblocks, strided, s);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return hipErrorInvalidValue;
}

// Tile counts of a Hartley pass (in place); returns its launch's blocks.
static int64_t dht_tiles(int L, DhtArgs& a) {
  switch (L) {
#define RSFDE_CASE(LL) \
  case LL:             \
    return dht_tiles_L<LL>(a);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return -1;
}

hipError_t launch_dht_tables(int L, int N, const cpx<double>* tw64, cpx<double>* chirp,
                             cpx<double>* khat, hipStream_t st) {
  switch (L) {
#define RSFDE_CASE(LL) \
  case LL:             \
    return launch_dht_tables_L<LL>(N, tw64, chirp, khat, st);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spectrum(int L, const double* s, int N, const cpx<double>* tw64, double* chat64,
                           float* chat32, double* q, hipStream_t st) {
  switch (L) {
#define RSFDE_CASE(LL) \
  case LL:             \
    return launch_spectrum_L<LL>(s, N, tw64, chat64, chat32, q, st);
    RSFDE_FOR_EACH_L(RSFDE_CASE)
#undef RSFDE_CASE
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
namespace {

thread_local hipError_t g_last_hip = hipSuccess;
thread_local char g_msg[256];

struct Axis {
  int N = 0, L = 0;
  double alpha = 0, h = 0, eta = 0;
  int64_t inner = 1;
  double *s = nullptr, *chat64 = nullptr, *q = nullptr, *lam64 = nullptr, *wq64 = nullptr;
  float *chat32 = nullptr, *lam32 = nullptr, *wq32 = nullptr;
  cpx<double>* tw64 = nullptr;
  cpx<float>* tw32 = nullptr;
  // Strang circulant form only: chirp (N), Bluestein kernel spectrum (L), Strang
  // eigenvalues of B and eta sigma / b (N each, Fourier order)
  cpx<double>*chirp = nullptr, *khat = nullptr;
  double *slam = nullptr, *swq = nullptr;
};

struct FieldHost {
  rsfde_field spec{};
  std::vector<double> amp;
  bool set = false;
  bool evaluated = false;  // time-independent field already in its buffer
};

struct Inst {
  rsfde_params p{};
  int d = 0;
  int64_t n = 0, nclo = 0, ldv = 0;
  int nb = 1;  // blocks of the Krylov sweeps and norms (kry_blocks, or kry_blocks_many on
               // handles of several instances, batched or not, so both agree bit for bit)
  Axis ax[3];
  double *e = nullptr, *f = nullptr, *F = nullptr, *b = nullptr, *V = nullptr;
  const double* ecur = nullptr;  // e of the current step (the caller's buffer or e)
  float* e32 = nullptr;
  void* tmp[4] = {nullptr, nullptr, nullptr, nullptr};
  GmresState* st = nullptr;
  unsigned* counters = nullptr;
  double* partial = nullptr;               // cycle-start norm and min/max partials
  double* pk[3] = {nullptr, nullptr, nullptr};  // CGS2 sweep partials (value-major)
  double* ebar = nullptr;
  double* eminmax = nullptr;
  bool ebar_set = false;
  double ebar_h = 0;
  double pscale = 1;
  // fields
  FieldHost fe, ff, fpsi;
  double* famp_e = nullptr;
  double* famp_f = nullptr;
  double* fmc = nullptr;
  double* fsin_e[3] = {nullptr, nullptr, nullptr};
  double* fsin_f[3] = {nullptr, nullptr, nullptr};
  double* fax[3] = {nullptr, nullptr, nullptr};  // per-axis factor tables (AX_ROWS x (N_i+2))
  // Arnoldi steps of the last cycle that ran at each cycle index of a step (the
  // first chunk of the next such cycle): the mixed form's two refinement sweeps
  // need different counts (about 5 and 6-7 on the benchmark grids)
  int k_prev[3] = {4, 4, 4};
  std::vector<hipGraphExec_t> gexec;  // captured Arnoldi steps: [2 j + (resolve pending)]
  const void* g_e = nullptr;           // e the captured steps read
  int var[3][2][2] = {};  // tile variant per axis, precision (FP64, FP32) and pass class
                          // (0: operator passes, 1: transform passes)
};

struct TimedPass {
  hipEvent_t a, b;
  double bytes;
  int cls;
  int step;   // Arnoldi step the launch belongs to (-1: not an Arnoldi step)
  bool spec;  // launched past the end of its cycle: exited on the status word
};

}  // namespace

#define CK(x)                          \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) {            \
      g_last_hip = e_;                 \
      return RSFDE_E_HIP;              \
    }                                  \
  } while (0)

#define CKS(x)                  \
  do {                          \
    int s_ = (x);               \
    if (s_ < 0) return s_;      \
  } while (0)

// one batched launch: the instances that share a pass position's transform
// length, precision, axis kind and tile shape
struct BGroup {
  int L = 0, var = 0;
  bool fp32 = false, strided = false;
  bool dht = false;             // Hartley passes (Strang form): ddesc instead of desc
  int op = 0;                   // (Hartley passes: DHT_PLAIN or DHT_SCALE)
  int ninst = 0;
  int64_t nblocks = 0;
  const BPass* desc = nullptr;  // device copies (batch descriptor buffer)
  const DBPass* ddesc = nullptr;
  const int* start = nullptr;
  int cls = 0;
  bool mv = false;  // operator pass (else sine transform); one op per group
  double bytes = 0;
};
struct BChain {
  std::vector<std::vector<BGroup>> pos;  // groups per pass position of the chain
};
struct KPlan {
  int ninst = 0;
  const KBatch* desc = nullptr;
  const int *start_nb = nullptr, *start_nbu = nullptr;
  int64_t nb_total = 0, nbu_total = 0;
  double vbytes = 0;  // one FP64 vector over all instances
  int m = 0;          // largest restart
};

struct BPlan {
  BChain rhs, resid, oper;
  KPlan kp;
  const FJob* fjobs = nullptr;
  const int* fstart = nullptr;
  int64_t fblocks = 0;
  int nf = 0;
};

struct RecPass {
  PassArgs a;
  bool fp32;
  int inst;
  bool stop_pend;  // runs before the step's resolve: stops on the pending step's status
  bool dht = false;  // a Hartley pass (Strang form): da and its launch's blocks dnb
  DhtArgs da{};
  int64_t dnb = 0;
};

struct rsfde_ctx {
  int count = 0;
  std::vector<Inst> inst;
  // graph replay of Arnoldi steps (rsfde_set_graph)
  bool graphs = false;
  hipStream_t cap = nullptr;             // private stream the steps are captured on
  std::vector<hipGraphExec_t> bgexec;    // batched steps captured on the full-set plan
  long long plan_gen = 0, bg_gen = -1;   // full-set plan generation the batched graphs belong to
  // batched engine (count > 1)
  bool batched = false;
  char* bdev = nullptr;          // descriptor buffer in the workspace
  char* bhost = nullptr;         // pinned staging copy
  size_t bcap = 0;
  struct Region {
    size_t base = 0, cap = 0, fill = 0;
  } rg[3];                       // 0: the step's full-set plan, 1: plans of later cycles, 2: field jobs
  GmresSummary* dsum = nullptr;  // gathered summaries (workspace) and their pinned copy
  GmresSummary* psum = nullptr;
  int* dmask = nullptr;          // per-slot "update may add V y" flags (workspace) and pinned copy
  int* pmask = nullptr;
  // cached full-set plan: valid while the u, e and f pointers of a step repeat
  BPlan full;
  bool full_valid = false;
  std::vector<const void*> full_key;
  std::vector<const void*> fjob_key;   // cached batched field-evaluation jobs
  int fjob_which = -1;
  int64_t fjob_blocks = 0;
  const FieldJob* fjob_dev = nullptr;
  const int* fjob_start = nullptr;
  std::vector<RecPass>* rec = nullptr;  // chain recording instead of launching
  int rec_inst = -1;
  bool rec_stop_pend = false;           // passes recorded now carry RecPass::stop_pend
  bool true_res = false;                 // rsfde_set_true_residual
  hipStream_t stream = nullptr;
  GmresSummary* pinned = nullptr;
  hipEvent_t sync_ev = nullptr;          // stream_wait's event (created on first use)
  unsigned tmask = 0;
  int tevery = 1;
  long long tseen[RSFDE_K_NCLASS] = {0};
  std::vector<TimedPass> pending;
  std::vector<hipEvent_t> ev_free;
  long long t_launches[RSFDE_K_NCLASS] = {0};
  double t_ms[RSFDE_K_NCLASS] = {0}, t_bytes[RSFDE_K_NCLASS] = {0};
  int cur_step = -1;  // Arnoldi step whose launches are being issued (timing tag)
};

static hipError_t get_event(rsfde_ctx* h, hipEvent_t* ev) {
  if (!h->ev_free.empty()) {
    *ev = h->ev_free.back();
    h->ev_free.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(ev);
}

// Launch `fn(ea, eb)` (returning hipError_t); when class `cls` is timed, the
// dispatch itself stamps the events (no extra stream commands).
template <typename Fn>
static int timed_launch(rsfde_ctx* h, int cls, double bytes, Fn fn) {
  if (((h->tmask >> cls) & 1u) && (h->tseen[cls]++ % h->tevery) == 0) {
    hipEvent_t ea, eb;
    CK(get_event(h, &ea));
    CK(get_event(h, &eb));
    CK(fn(ea, eb));
    h->pending.push_back(TimedPass{ea, eb, bytes, cls, h->cur_step, false});
  } else {
    CK(fn(nullptr, nullptr));
  }
  return RSFDE_OK;
}

// ---------------------------------------------------------------------------
// validation and layout
// ---------------------------------------------------------------------------
static int validate(const rsfde_params* p) {
  if (!p) return RSFDE_E_INVALID_ARG;
  if (p->d < 1 || p->d > 3) return RSFDE_E_INVALID_ARG;
  double ksum = 0.0;
  int64_t n = 1;
  for (int i = 0; i < p->d; ++i) {
    if (p->n[i] < 1 || p->n[i] > 100000) return RSFDE_E_INVALID_ARG;
    if (!(p->lo[i] < p->hi[i]) || !isfinite(p->lo[i]) || !isfinite(p->hi[i])) return RSFDE_E_INVALID_ARG;
    if (!(p->alpha[i] > 1.0 && p->alpha[i] < 2.0)) return RSFDE_E_INVALID_ARG;
    if (!(p->kappa[i] >= 0.0) || !isfinite(p->kappa[i])) return RSFDE_E_INVALID_ARG;
    ksum += p->kappa[i];
    n *= p->n[i];
  }
  if (!(ksum > 0.0)) return RSFDE_E_INVALID_ARG;
  if (!(p->dt > 0.0) || !isfinite(p->dt)) return RSFDE_E_INVALID_ARG;
  const bool eunset = p->e_min == 0.0 && p->e_max == 0.0;
  if (!eunset && !(p->e_min > 0.0 && p->e_min <= p->e_max && isfinite(p->e_max))) return RSFDE_E_INVALID_ARG;
  if (p->restart < 1 || p->restart > RSFDE_MAX_RESTART) return RSFDE_E_INVALID_ARG;
  if (!(p->rtol > 0.0) || !(p->rtol < 1.0)) return RSFDE_E_INVALID_ARG;
  if (p->max_cycles < 1) return RSFDE_E_INVALID_ARG;
  if (p->precision != RSFDE_FP64 && p->precision != RSFDE_MIXED) return RSFDE_E_INVALID_ARG;
  if (p->x0_mode != 0 && p->x0_mode != 1) return RSFDE_E_INVALID_ARG;
  if (!(p->inner_rtol >= 0.0 && p->inner_rtol < 1.0)) return RSFDE_E_INVALID_ARG;
  if (p->max_outer < 0) return RSFDE_E_INVALID_ARG;
  if (!(p->outer_rtol >= 0.0 && p->outer_rtol <= p->rtol)) return RSFDE_E_INVALID_ARG;
  if (p->method != RSFDE_OPGM && p->method != RSFDE_TPGM && p->method != RSFDE_SPGM)
    return RSFDE_E_INVALID_ARG;
  if (p->method != RSFDE_OPGM && p->precision != RSFDE_FP64) return RSFDE_E_UNSUPPORTED;
  if (n > ((int64_t)1 << 34)) return RSFDE_E_INVALID_ARG;
  for (int i = 0; i < p->d; ++i) {
    const int64_t L = 2 * (p->n[i] + 1);
    if (L > 4096 || !supported_L((int)L)) return RSFDE_E_UNSUPPORTED;
  }
  return RSFDE_OK;
}

struct Bump {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* ptr = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return ptr;
  }
};

static void layout(Inst& I, Bump& B) {
  const rsfde_params& p = I.p;
  I.d = p.d;
  I.n = 1;
  I.nclo = 1;
  for (int i = 0; i < p.d; ++i) {
    I.n *= p.n[i];
    I.nclo *= p.n[i] + 2;
  }
  I.ldv = (I.n + 63) / 64 * 64;
  I.st = B.take<GmresState>(1);
  I.counters = B.take<unsigned>(64);
  I.partial = B.take<double>((size_t)4096);
  for (int k = 0; k < 3; ++k) I.pk[k] = B.take<double>((size_t)RSFDE_PVS * (RSFDE_MAX_RESTART + 1));
  I.ebar = B.take<double>(1);
  I.eminmax = B.take<double>(2);
  for (int i = 0; i < p.d; ++i) {
    Axis& A = I.ax[i];
    A.N = (int)p.n[i];
    A.L = 2 * (A.N + 1);
    A.s = B.take<double>(A.N);
    A.q = B.take<double>(A.N);
    A.lam64 = B.take<double>(A.N);
    A.wq64 = B.take<double>(A.N);
    A.chat64 = B.take<double>(A.L);
    A.lam32 = B.take<float>(A.N);
    A.wq32 = B.take<float>(A.N);
    A.chat32 = B.take<float>(A.L);
    A.tw64 = B.take<cpx<double>>(A.L);
    A.tw32 = B.take<cpx<float>>(A.L);
    if (p.method == RSFDE_SPGM) {
      A.chirp = B.take<cpx<double>>(A.N);
      A.khat = B.take<cpx<double>>(A.L);
      A.slam = B.take<double>(A.N);
      A.swq = B.take<double>(A.N);
    }
  }
  I.e = B.take<double>(I.n);
  if (p.precision == RSFDE_MIXED) I.e32 = B.take<float>(I.n);
  I.f = B.take<double>(I.nclo);
  I.F = B.take<double>(I.n);
  I.b = B.take<double>(I.n);
  for (int k = 0; k < 4; ++k) I.tmp[k] = B.take<double>(I.n);
  I.V = B.take<double>((size_t)(p.restart + 1) * I.ldv);
  I.famp_e = B.take<double>(512);
  I.famp_f = B.take<double>(512);
  I.fmc = B.take<double>(3 * RSFDE_MC_STRIDE);
  for (int i = 0; i < p.d; ++i) {
    I.fsin_e[i] = B.take<double>((size_t)RSFDE_MAXMODES * (p.n[i] + 2));
    I.fsin_f[i] = B.take<double>((size_t)RSFDE_MAXMODES * (p.n[i] + 2));
    I.fax[i] = B.take<double>((size_t)AX_ROWS * (p.n[i] + 2));
  }
}

// ---------------------------------------------------------------------------
// pass chains
// ---------------------------------------------------------------------------
static PassArgs mk_pass(const Inst& I, int axis, int op, bool fp32) {
  PassArgs a;
  memset(&a, 0, sizeof(a));
  const Axis& A = I.ax[axis];
  a.op = op;
  a.N = A.N;
  a.d = I.d;
  a.axis = axis;
  int64_t inner = 1;
  for (int l = 0; l < axis; ++l) inner *= I.ax[l].N;
  a.inner = inner;
  a.npencil = I.n / A.N;
  int nt, ppt;
  a.var = I.var[axis][fp32 ? 1 : 0][op <= OP_MV_LAST ? 0 : 1];
  pass_shape_rt(A.L, fp32, axis > 0, a.var, &nt, &ppt);
  if (axis == 0) {
    a.tiles_inner = 1;
    a.ntiles = (a.npencil + ppt - 1) / ppt;
    a.xcd_remap = 0;
    a.nlaunch = a.ntiles;
  } else {
    a.tiles_inner = (inner + ppt - 1) / ppt;
    a.ntiles = (a.npencil / inner) * a.tiles_inner;
    a.xcd_remap = 1;
    a.nlaunch = (a.ntiles + 7) / 8 * 8;
  }
  a.bd = 1.0 - A.alpha / 12.0;
  a.bo = A.alpha / 24.0;
  a.eta = A.eta;
  a.gam = 1.0;
  a.xcoef = 0.0;
  a.chat = fp32 ? (const void*)A.chat32 : (const void*)A.chat64;
  a.tw = fp32 ? (const void*)A.tw32 : (const void*)A.tw64;
  for (int l = 0; l < 3; ++l) {
    a.Nax[l] = l < I.d ? I.ax[l].N : 1;
    a.lam[l] = l < I.d ? (fp32 ? (const void*)I.ax[l].lam32 : (const void*)I.ax[l].lam64) : nullptr;
    a.wq[l] = l < I.d ? (fp32 ? (const void*)I.ax[l].wq32 : (const void*)I.ax[l].wq64) : nullptr;
  }
  a.ebar = I.ebar;
  a.pscale = I.pscale;
  return a;
}

static double pass_bytes(const PassArgs& a, const Inst& I, bool fp32) {
  const double w = fp32 ? 4.0 : 8.0;
  const double n = (double)I.n;
  const double cin = (a.flags & FL_IN64) ? 8.0 : w;
  const double aout = (a.flags & FL_OUT64) ? 8.0 : w;
  switch (a.op) {
    case OP_MV_FIRST:
      return n * (cin + w + 2 * w);
    case OP_MV_MID:
      return n * 4 * w;
    case OP_MV_LAST: {
      double b = n * (cin + w + aout);  // Toeplitz input, stencil input (a or e), output
      if (a.in_x) b += n * 8.0;
      return b;
    }
    default:
      return n * (cin + aout);
  }
}

static int op_class(int op) {
  switch (op) {
    case OP_MV_FIRST: return RSFDE_K_MV_FIRST;
    case OP_MV_MID: return RSFDE_K_MV_MID;
    case OP_MV_LAST: return RSFDE_K_MV_LAST;
    case OP_DST: return RSFDE_K_DST;
    default: return RSFDE_K_DSD;
  }
}

static int run_pass(rsfde_ctx* h, const Inst& I, const PassArgs& a, bool fp32) {
  const int L = I.ax[a.axis].L;
  if (h->rec) {
    h->rec->push_back(RecPass{a, fp32, h->rec_inst, h->rec_stop_pend});
    return RSFDE_OK;
  }
  if (a.ntiles <= 0) return RSFDE_OK;
  if (a.nlaunch > 0x7fffffffLL) return RSFDE_E_UNSUPPORTED;
  return timed_launch(h, op_class(a.op), pass_bytes(a, I, fp32), [&](hipEvent_t ea, hipEvent_t eb) {
    return launch_pass(L, fp32, a, a.axis > 0, h->stream, ea, eb);
  });
}

// Timed launches of Arnoldi steps >= kend ran past the end of their cycle (the
// host launches chunks of steps speculatively; such kernels exit on the status
// word): they are left out of the timing.
static void mark_speculative(rsfde_ctx* h, int kend) {
  for (auto& tp : h->pending)
    if (tp.step >= kend) tp.spec = true;
}

static int flush_timing(rsfde_ctx* h) {
  for (auto& tp : h->pending) {
    if (!tp.spec) {
      float ms = 0.f;
      CK(hipEventSynchronize(tp.b));
      CK(hipEventElapsedTime(&ms, tp.a, tp.b));
      h->t_ms[tp.cls] += ms;
      h->t_bytes[tp.cls] += tp.bytes;
      h->t_launches[tp.cls] += 1;
    }
    h->ev_free.push_back(tp.a);
    h->ev_free.push_back(tp.b);
  }
  h->pending.clear();
  return RSFDE_OK;
}

// Transform, diagonal scaling (PM_*), transform for an FP64 r: (BP)^{-1} r, or
// a factor of the two-sided form.  Temporaries T[0], T[1], T[2], T[3] in turn
// (d = 3); out may be T[2], r may be T[3].  accum: the result is added to out.
static int run_prec(rsfde_ctx* h, const Inst& I, bool fp32, const double* r, double* out,
                    int pmode = PM_BP_INV, const int* stop_fl = nullptr,
                    void* const* temps = nullptr, bool accum = false) {
  const int d = I.d;
  void* const* T = temps ? temps : I.tmp;
  const int acc = accum ? FL_ACCUM : 0;
  if (d == 1) {
    PassArgs t = mk_pass(I, 0, OP_DSD, fp32);
    t.flags = FL_IN64 | FL_OUT64 | acc;
    t.in_c = r;
    t.out_a = out;
    t.pmode = pmode;
    t.stop_fl = stop_fl;
    return run_pass(h, I, t, fp32);
  }
  int cur = -1;
  for (int ax = d - 1; ax >= 1; --ax) {
    PassArgs t = mk_pass(I, ax, OP_DST, fp32);
    t.flags = cur < 0 ? FL_IN64 : 0;
    t.in_c = cur < 0 ? (const void*)r : T[cur];
    const int o = cur < 0 ? 0 : (cur + 1) & 3;
    t.out_a = T[o];
    t.stop_fl = stop_fl;
    CKS(run_pass(h, I, t, fp32));
    cur = o;
  }
  {
    PassArgs t = mk_pass(I, 0, OP_DSD, fp32);
    t.in_c = T[cur];
    const int o = (cur + 1) & 3;
    t.out_a = T[o];
    t.pmode = pmode;
    t.stop_fl = stop_fl;
    CKS(run_pass(h, I, t, fp32));
    cur = o;
  }
  for (int ax = 1; ax <= d - 1; ++ax) {
    PassArgs t = mk_pass(I, ax, OP_DST, fp32);
    t.in_c = T[cur];
    const bool last = ax == d - 1;
    const int o = (cur + 1) & 3;
    t.flags = last ? FL_OUT64 | acc : 0;
    t.out_a = last ? (void*)out : T[o];
    t.stop_fl = stop_fl;
    CKS(run_pass(h, I, t, fp32));
    cur = o;
  }
  return RSFDE_OK;
}

// (ebar c(B) + c(S))^{-1} r of the Strang circulant form: Hartley passes along
// axes d-1..1, Hartley / 1/m / Hartley along axis 0, Hartley along axes 1..d-1.
// r is the temporary T[ri] (or any FP64 vector with ri = -1); the passes use the
// temporaries after it in turn, and the last one writes out.
static int run_strang_prec(rsfde_ctx* h, const Inst& I, const double* r, int ri, double* out,
                           const int* stop_fl = nullptr) {
  const int d = I.d;
  void* const* T = I.tmp;
  double pscale = 1.0;
  for (int l = 0; l < d; ++l) pscale /= (double)I.ax[l].N;
  auto mk = [&](int axis, int op) {
    DhtArgs a;
    memset(&a, 0, sizeof(a));
    const Axis& A = I.ax[axis];
    a.op = op;
    a.N = A.N;
    a.d = d;
    a.axis = axis;
    int64_t inner = 1;
    for (int l = 0; l < axis; ++l) inner *= I.ax[l].N;
    a.inner = inner;
    a.npencil = I.n / A.N;
    a.chirp = A.chirp;
    a.khat = A.khat;
    a.tw = A.tw64;
    for (int l = 0; l < 3; ++l) {
      a.Nax[l] = l < d ? I.ax[l].N : 1;
      a.lam[l] = l < d ? I.ax[l].slam : nullptr;
      a.wq[l] = l < d ? I.ax[l].swq : nullptr;
    }
    a.ebar = I.ebar;
    a.pscale = pscale;
    a.stop_fl = stop_fl;
    return a;
  };
  auto launch = [&](const DhtArgs& a, const void* in, double* o) -> int {
    DhtArgs b = a;
    b.in = (const double*)in;
    b.out = o;
    const int L = I.ax[b.axis].L;
    if (h->rec) {
      RecPass rp;
      memset(&rp.a, 0, sizeof(rp.a));
      rp.a.axis = b.axis;
      rp.fp32 = false;
      rp.inst = h->rec_inst;
      rp.stop_pend = false;
      rp.dht = true;
      rp.dnb = dht_tiles(L, b);
      rp.da = b;
      if (rp.dnb < 0 || rp.dnb > 0x7fffffffLL) return RSFDE_E_UNSUPPORTED;
      h->rec->push_back(rp);
      return RSFDE_OK;
    }
    return timed_launch(h, b.op == DHT_SCALE ? RSFDE_K_DSD : RSFDE_K_DST, 16.0 * (double)I.n,
                        [&](hipEvent_t ea, hipEvent_t eb) -> hipError_t {
                          if (ea) {
                            hipError_t e = hipEventRecord(ea, h->stream);
                            if (e != hipSuccess) return e;
                          }
                          hipError_t e = launch_dht(L, b, h->stream);
                          if (e == hipSuccess && eb) e = hipEventRecord(eb, h->stream);
                          return e;
                        });
  };
  if (d == 1) return launch(mk(0, DHT_SCALE), r, out);
  int cur = ri;
  const void* src = r;
  auto next = [&]() { return cur < 0 ? 0 : (cur + 1) & 3; };
  for (int ax = d - 1; ax >= 1; --ax) {
    const int o = next();
    CKS(launch(mk(ax, DHT_PLAIN), src, (double*)T[o]));
    cur = o;
    src = T[o];
  }
  {
    const int o = next();
    CKS(launch(mk(0, DHT_SCALE), src, (double*)T[o]));
    cur = o;
    src = T[o];
  }
  for (int ax = 1; ax <= d - 1; ++ax) {
    const bool last = ax == d - 1;
    const int o = next();
    CKS(launch(mk(ax, DHT_PLAIN), src, last ? out : (double*)T[o]));
    cur = o;
    src = T[o];
  }
  return RSFDE_OK;
}

enum Chain { CH_APPLY_A = 0, CH_RHS = 1, CH_RESID = 2, CH_OPER = 3, CH_R0 = 4 };

// Operator chains along the axes (x_1 first).  CH_APPLY_A: out = A x.
// CH_RHS: out = B E x - S x + xcoef * xin.  CH_RESID: out = M (xin - A x).
// CH_R0: out = M (xcoef * xin - 2 S x), the step's first residual
// M (b - A u^{(m)}) with b = (B E - S) u^{(m)} + dt F written out (the B E terms
// cancel), one-sided form only.
// CH_OPER: out = M A (sc * x).  M = (BP)^{-1} in the one-sided form; in the
// two-sided form (eq. Pls) M = P^{-1/2} B^{-1} and CH_OPER first takes x to
// P^{-1/2} x (into T[2]; the step's scale is applied when the next pass reads
// it).  x is FP64; out is FP64.
static int run_chain(rsfde_ctx* h, const Inst& I, int kind, bool fp32, const double* x,
                     const double* sc, const double* xin, double xcoef, double* out,
                     const GmRes* gm = nullptr, const int* stop_fl = nullptr) {
  const int d = I.d;
  const void* e = fp32 ? (const void*)I.e32 : (const void*)I.ecur;
  const bool strang = I.p.method == RSFDE_SPGM && (kind == CH_RESID || kind == CH_OPER);
  // the tau preconditioner fused into the operator passes (not in the Strang form,
  // whose solve follows the operator as its own chain from a temporary)
  const bool prec = (kind == CH_RESID || kind == CH_OPER || kind == CH_R0) && !strang;
  const int st_i = d == 3 ? 0 : 3;  // Strang form: temporary between the two chains
  double* const op_out = strang ? (double*)I.tmp[st_i] : out;
  const bool two = I.p.method == RSFDE_TPGM;
  const int pm = two ? PM_PH_BINV : PM_BP_INV;
  if (two && kind == CH_OPER) {
    // runs before the step's resolve: exit on the status before the pending step
    const int* pre_stop = gm ? &I.st->FL[gm->pend >= 0 ? gm->pend : gm->j] : stop_fl;
    h->rec_stop_pend = gm != nullptr;
    const int pre_status = run_prec(h, I, fp32, x, (double*)I.tmp[2], PM_PH, pre_stop);
    h->rec_stop_pend = false;
    CKS(pre_status);
    x = (const double*)I.tmp[2];
  }
  const double sgn = kind == CH_RHS ? -1.0 : 1.0;
  const double gam = kind == CH_RESID ? -1.0 : (kind == CH_R0 ? -2.0 : 1.0);
  const int no_e = kind == CH_R0 ? FL_NO_E : 0;
  void* const* T = I.tmp;
  if (d == 1) {
    PassArgs a = mk_pass(I, 0, OP_MV_LAST, fp32);
    a.flags = FL_FIRST_IS_LAST | FL_IN64 | FL_OUT64 | (prec ? FL_PREC_FULL : 0) | no_e;
    a.pmode = pm;
    a.in_c = x;
    a.sc_ptr = sc;
    a.in_a = e;
    a.eta = sgn * I.ax[0].eta;
    a.gam = gam;
    a.in_x = xin;
    a.xcoef = xcoef;
    a.out_a = op_out;
    if (gm) {
      a.use_gm = 1;
      a.gm = *gm;
      a.sc_ptr = nullptr;
    }
    CKS(run_pass(h, I, a, fp32));
    if (strang) return run_strang_prec(h, I, op_out, st_i, out, stop_fl);
    return RSFDE_OK;
  }
  // first axis
  PassArgs a = mk_pass(I, 0, OP_MV_FIRST, fp32);
  a.flags = FL_IN64 | no_e;
  a.in_c = x;
  a.sc_ptr = sc;
  a.in_a = e;
  a.eta = sgn * I.ax[0].eta;
  a.out_a = T[0];
  a.out_c = T[1];
  if (gm) {
    a.use_gm = 1;
    a.gm = *gm;
    a.sc_ptr = nullptr;
  }
  CKS(run_pass(h, I, a, fp32));
  int ia = 0, ic = 1;
  if (d == 3) {
    PassArgs m = mk_pass(I, 1, OP_MV_MID, fp32);
    m.in_a = T[0];
    m.in_c = T[1];
    m.eta = sgn * I.ax[1].eta;
    m.out_a = T[2];
    m.out_c = T[3];
    m.stop_fl = stop_fl;
    CKS(run_pass(h, I, m, fp32));
    ia = 2;
    ic = 3;
  }
  PassArgs z = mk_pass(I, d - 1, OP_MV_LAST, fp32);
  z.in_a = T[ia];
  z.in_c = T[ic];
  z.eta = sgn * I.ax[d - 1].eta;
  z.gam = gam;
  z.in_x = xin;
  z.xcoef = xcoef;
  z.stop_fl = stop_fl;
  if (!prec) {
    z.flags = FL_OUT64;
    z.out_a = op_out;
    CKS(run_pass(h, I, z, fp32));
    if (strang) return run_strang_prec(h, I, op_out, st_i, out, stop_fl);
    return RSFDE_OK;
  }
  z.flags = FL_DST_AFTER;
  int cur = d == 2 ? 2 : 0;  // holds the transformed w
  z.out_a = T[cur];
  CKS(run_pass(h, I, z, fp32));
  // remaining forward transforms on axes d-2 .. 1, scaling pass on axis 0,
  // inverse transforms on axes 1 .. d-1
  auto nxt = [&](int c) { return (c + 1) & 3; };
  for (int ax = d - 2; ax >= 1; --ax) {
    PassArgs t = mk_pass(I, ax, OP_DST, fp32);
    t.in_c = T[cur];
    t.out_a = T[nxt(cur)];
    t.stop_fl = stop_fl;
    CKS(run_pass(h, I, t, fp32));
    cur = nxt(cur);
  }
  {
    PassArgs t = mk_pass(I, 0, OP_DSD, fp32);
    t.in_c = T[cur];
    t.out_a = T[nxt(cur)];
    t.stop_fl = stop_fl;
    t.pmode = pm;
    CKS(run_pass(h, I, t, fp32));
    cur = nxt(cur);
  }
  for (int ax = 1; ax <= d - 1; ++ax) {
    PassArgs t = mk_pass(I, ax, OP_DST, fp32);
    t.in_c = T[cur];
    t.stop_fl = stop_fl;
    const bool last = ax == d - 1;
    t.flags = last ? FL_OUT64 : 0;
    t.out_a = last ? (void*)out : T[nxt(cur)];
    CKS(run_pass(h, I, t, fp32));
    cur = nxt(cur);
  }
  return RSFDE_OK;
}

// ---------------------------------------------------------------------------
// fields
// ---------------------------------------------------------------------------
static FieldDev field_dev(const Inst& I, const FieldHost& F, bool is_e) {
  FieldDev fd;
  memset(&fd, 0, sizeof(fd));
  fd.kind = F.set ? F.spec.kind : RSFDE_FIELD_ZERO;
  for (int k = 0; k < 4; ++k) fd.c[k] = F.spec.c[k];
  fd.K = F.spec.modes;
  fd.a = (int)llround(F.spec.c[1]);
  double nrm = 0;
  for (double v : F.amp) nrm += fabs(v);
  fd.norm = nrm > 0 ? nrm : 1.0;
  fd.amp = is_e ? I.famp_e : I.famp_f;
  for (int i = 0; i < 3; ++i) fd.sintab[i] = i < I.d ? (is_e ? I.fsin_e[i] : I.fsin_f[i]) : nullptr;
  fd.mc = I.fmc;
  for (int i = 0; i < 3; ++i) fd.ax[i] = i < I.d ? I.fax[i] : nullptr;
  return fd;
}

static GridDev grid_dev(const Inst& I, bool closure) {
  GridDev g;
  memset(&g, 0, sizeof(g));
  g.d = I.d;
  g.closure = closure ? 1 : 0;
  for (int i = 0; i < I.d; ++i) {
    g.N[i] = I.ax[i].N;
    g.lo[i] = I.p.lo[i];
    g.h[i] = I.ax[i].h;
    g.kappa[i] = I.p.kappa[i];
    g.inv[i] = 1.0 / (double)(closure ? I.ax[i].N + 2 : I.ax[i].N);
  }
  g.size = closure ? I.nclo : I.n;
  return g;
}

static int eval_field(rsfde_ctx* h, Inst& I, int which, double t, double* out) {
  FieldDev fe = field_dev(I, I.fe, true);
  FieldDev ff = field_dev(I, which == RSFDE_WHICH_PSI ? I.fpsi : I.ff, false);
  if (which == RSFDE_WHICH_PSI) {
    ff.a = (int)llround(I.fpsi.spec.c[1]);
  }
  CK(fields_eval(fe, ff, which, grid_dev(I, which == RSFDE_WHICH_F), t, out, h->stream));
  return RSFDE_OK;
}

// ---------------------------------------------------------------------------
// one step of one instance
// ---------------------------------------------------------------------------
// Wait for the stream's work enqueued so far by spinning on an event query.  The
// read of a chunk's status is on the critical path (the GPU idles until the
// host launches what follows), and a blocking synchronisation adds the host
// thread's wake-up latency to that idle time.
static hipError_t stream_wait(rsfde_ctx* h) {
  static const bool blocking = [] {
    const char* e = getenv("RSFDE_BLOCKING_SYNC");
    return e && atoi(e) != 0;
  }();
  if (blocking) return hipStreamSynchronize(h->stream);
  if (!h->sync_ev) {
    const hipError_t e = hipEventCreateWithFlags(&h->sync_ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipEventRecord(h->sync_ev, h->stream);
  if (e != hipSuccess) return e;
  while ((e = hipEventQuery(h->sync_ev)) == hipErrorNotReady) {
  }
  return e;
}

static int read_summary(rsfde_ctx* h, const Inst& I, GmresSummary* out) {
  CK(hipMemcpyAsync(h->pinned, &I.st->sum, sizeof(GmresSummary), hipMemcpyDeviceToHost, h->stream));
  CK(stream_wait(h));
  *out = *h->pinned;
  if (!h->pending.empty()) {
    if (out->flag != GM_RUNNING) mark_speculative(h, out->k);
    CKS(flush_timing(h));
  }
  return RSFDE_OK;
}

// Steps still to launch after a chunk that ended at step j_done with the cycle
// running: the least-squares residual has fallen from beta (cycle start) to res
// in j_done steps; at the same geometric rate it reaches thr after
// log(thr/res)/log(rate) more.  One step when the rate says nothing (stagnation).
static int next_chunk(const GmresSummary& S, int j_done, int left) {
  if (left <= 1 || j_done <= 0 || !(S.beta > 0.0) || !(S.res > 0.0) || !(S.thr > 0.0)) return 1;
  const double rate = pow(S.res / S.beta, 1.0 / j_done);
  if (!(rate > 0.0 && rate < 0.95)) return 1;
  const double need = ceil(log(S.thr / S.res) / log(rate));
  if (!(need >= 1.0)) return 1;
  return need >= (double)left ? left : (int)need;
}

// Runs one GMRES cycle's iterations after cycle_init, launched in chunks
// without host synchronisation inside a chunk: the chunk length is the previous
// cycle's iteration count, then the steps the residual's rate of decrease
// predicts (next_chunk).  Kernels of steps past convergence exit on the device
// status (FL); the update kernel that closes a chunk resolves its last step and
// adds V y once the cycle has finished.
// Replay of one Arnoldi step from a graph captured on the private stream: the
// step's launches have fixed arguments for a given (j, pending resolve), so
// they are captured once and replayed on the handle's stream.  Used when graph
// replay is on and no kernel class is being timed (event-stamped dispatches stay
// outside graphs).
template <typename Fn>
static int graph_step(rsfde_ctx* h, std::vector<hipGraphExec_t>& cache, size_t slot, Fn launch) {
  if (cache.size() <= slot) cache.resize(slot + 1, nullptr);
  if (!cache[slot]) {
    hipStream_t saved = h->stream;
    h->stream = h->cap;
    CK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    const int st = launch();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &g);
    h->stream = saved;
    if (st < 0) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    CK(e);
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CK(ei);
    cache[slot] = x;
  }
  CK(hipGraphLaunch(cache[slot], h->stream));
  return RSFDE_OK;
}

static void graphs_clear(std::vector<hipGraphExec_t>& cache) {
  for (auto& x : cache)
    if (x) (void)hipGraphExecDestroy(x);
  cache.clear();
}

static int run_cycle(rsfde_ctx* h, Inst& I, bool fp32, double* x, GmresSummary* S, int cyc) {
  const int m = I.p.restart;
  const int nb = I.nb;
  int j = 0;
  int pending = -1;  // step the next first pass must resolve (-1: already resolved)
  int chunk = std::max(1, std::min(m, I.k_prev[std::min(cyc, 2)]));
  while (true) {
    const int jend = std::min(m, j + chunk);
    for (int jj = j; jj < jend; ++jj) {
      const int pend = jj == j ? pending : jj - 1;
      auto launch = [&]() -> int {
        h->cur_step = jj;
        double* vj = I.V + (int64_t)jj * I.ldv;
        double* w = I.V + (int64_t)(jj + 1) * I.ldv;
        GmRes g;
        g.st = I.st;
        g.p3 = I.pk[2];
        g.nb3 = nb;
        g.j = jj;
        g.pend = pend;
        g.m = m;
        CKS(run_chain(h, I, CH_OPER, fp32, vj, nullptr, nullptr, 0.0, w, &g, &I.st->FL[jj]));
        KryArgs ka;
        ka.V = I.V;
        ka.ldv = I.ldv;
        ka.n = I.n;
        ka.w = w;
        ka.st = I.st;
        ka.pa = I.pk[0];
        ka.pb = I.pk[1];
        ka.pc = I.pk[2];
        ka.j = jj;
        ka.m = m;
        ka.nb = nb;
        const double vb = 8.0 * (double)I.n;
        CKS(timed_launch(h, RSFDE_K_DOTS, vb * (jj + 2),
                         [&](hipEvent_t ea, hipEvent_t eb) { return kry_sweep(1, ka, h->stream, ea, eb); }));
        // sweep B reads columns 0..j and w, writes column j (j >= 1) and w
        CKS(timed_launch(h, RSFDE_K_ORTH_DOTS, vb * (jj + 2 + (jj >= 1 ? 2 : 1)),
                         [&](hipEvent_t ea, hipEvent_t eb) { return kry_sweep(2, ka, h->stream, ea, eb); }));
        h->cur_step = -1;
        return RSFDE_OK;
      };
      if (h->graphs && h->tmask == 0) {
        const void* ek = fp32 ? (const void*)I.e32 : (const void*)I.ecur;
        if (ek != I.g_e) {
          graphs_clear(I.gexec);
          I.g_e = ek;
        }
        CKS(graph_step(h, I.gexec, (size_t)(2 * jj + (pend >= 0 ? 1 : 0)), launch));
      } else {
        CKS(launch());
      }
    }
    GmRes gu;
    gu.st = I.st;
    gu.p3 = I.pk[2];
    gu.nb3 = nb;
    gu.j = jend - 1;
    gu.pend = jend - 1;
    gu.m = m;
    // two-sided form: the update V y is written to T[3] and u += P^{-1/2} (V y)
    // once the cycle has ended (the last pass of the factor adds into u)
    const bool two = I.p.method == RSFDE_TPGM;
    double* xu = two ? (double*)I.tmp[3] : x;
    CKS(timed_launch(h, RSFDE_K_UPDATE, 0.0, [&](hipEvent_t ea, hipEvent_t eb) {
      return kry_update(I.V, I.ldv, I.n, xu, gu, h->stream, ea, eb, two ? 1 : 0);
    }));
    CKS(read_summary(h, I, S));
    if (S->flag != GM_RUNNING) {
      if (two && S->flag != GM_NONFINITE && S->k > 0)
        CKS(run_prec(h, I, fp32, xu, x, PM_PH, nullptr, nullptr, true));
      return RSFDE_OK;
    }
    j = jend;
    pending = -1;
    chunk = next_chunk(*S, j, m - j);
    if (j >= m) return RSFDE_OK;  // cannot happen: the last step of a cycle is never running
  }
}

// Bound on the FP64 preconditioned true residual that ends the mixed form's
// refinement, relative to ||z_0||: a tenth of rtol unless set.  Two solutions
// that both meet rtol may differ by about cond * rtol; refining a decade further
// keeps the refined solution well inside the FP64 solve's own distance from the
// exact solution of the step's system.
static double outer_tol(const rsfde_params& p) { return p.outer_rtol > 0.0 ? p.outer_rtol : 0.1 * p.rtol; }

// Tolerance of each FP32 inner solve of the mixed form, relative to its start:
// unless set, the square root of the outer bound (two refinement sweeps reach
// it), kept within [1e-6, 1e-3] (below 1e-6 the FP32 operator's rounding, not
// the inner tolerance, limits what a sweep gains).
static double inner_tol(const rsfde_params& p) {
  if (p.inner_rtol > 0.0) return p.inner_rtol;
  return std::min(1e-3, std::max(1e-6, std::sqrt(outer_tol(p))));
}

static int step_one(rsfde_ctx* h, Inst& I, const double* e_half, const double* f_half, double* u,
                    rsfde_stats* stats) {
  if (!I.ebar_set) return RSFDE_E_STATE;
  if ((uintptr_t)u & 15) return RSFDE_E_INVALID_ARG;
  const rsfde_params& p = I.p;
  const bool mixed = p.precision == RSFDE_MIXED;
  I.ecur = e_half;  // read in place (no copy)
  GridDev gi = grid_dev(I, false);
  double al[3] = {I.p.alpha[0], I.p.alpha[1], I.p.alpha[2]};
  CK(compute_F(f_half, gi, al, I.F, h->stream));
  if (mixed) CK(convert_f64_f32(I.ecur, I.e32, I.n, h->stream));
  // One-sided FP64 steps from u^(m) (d >= 2) start from M (dt F - 2 S u^(m)), which
  // is M (b - A u^(m)) without forming b; b itself is formed from the copy of u^(m)
  // kept in its buffer only when a restart or the true-residual check needs it.
  // Handles of several instances keep forming b first, as their batched launches
  // do, so that batched and one-at-a-time steps of a handle agree bit for bit.
  const bool r0_path =
      !mixed && p.x0_mode == 0 && p.method == RSFDE_OPGM && I.d >= 2 && h->count == 1;
  bool have_b = !r0_path;
  auto need_b = [&]() -> int {
    if (!have_b) {
      // b = (B E - S) u^(m) + dt F from the copy in I.b, written over it (the chain's
      // first pass reads I.b before its last pass writes it)
      CKS(run_chain(h, I, CH_RHS, false, I.b, nullptr, I.F, p.dt, I.b));
      have_b = true;
    }
    return RSFDE_OK;
  };
  if (r0_path) {
    CK(hipMemcpyAsync(I.b, u, (size_t)I.n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  } else {
    // b = (B E - S) u + dt F
    CKS(run_chain(h, I, CH_RHS, false, u, nullptr, I.F, p.dt, I.b));
  }
  if (p.x0_mode == 1) CK(fill_f64(u, I.n, 0.0, h->stream));
  rsfde_stats st;
  memset(&st, 0, sizeof(st));
  GmresSummary S;
  memset(&S, 0, sizeof(S));
  const double inner_rtol = inner_tol(p);
  const double stop_rtol = mixed ? outer_tol(p) : p.rtol;
  const int max_outer = p.max_outer > 0 ? p.max_outer : 30;
  const int max_loops = mixed ? max_outer + 1 : p.max_cycles;
  int status = RSFDE_W_NOT_CONVERGED;
  double true_res = -1.0;
  for (int cyc = 0; cyc < max_loops; ++cyc) {
    // z = (BP)^{-1} (b - A u) in FP64 into V_0
    if (cyc == 0 && r0_path) {
      CKS(run_chain(h, I, CH_R0, false, u, nullptr, I.F, p.dt, I.V));
    } else {
      CKS(need_b());
      CKS(run_chain(h, I, CH_RESID, false, u, nullptr, I.b, 1.0, I.V));
    }
    CK(kry_cycle_init(I.V, I.n, I.nb, I.st, I.partial, cyc == 0 ? 1 : 0, stop_rtol, inner_rtol,
                      mixed ? 1 : 0, p.restart, h->stream));
    if (mixed && cyc == max_outer) {
      // final check only
      CKS(read_summary(h, I, &S));
      if (S.flag == GM_CONVERGED) status = RSFDE_OK;
      break;
    }
    if (mixed && cyc > 0) {
      // a refinement sweep's start usually finds the FP64 residual below the bound
      // already (the previous inner solve reached it): read the start's status
      // before launching steps, which would otherwise run a whole chunk of
      // speculative steps that exit only after loading their tiles
      CKS(read_summary(h, I, &S));
      if (S.flag == GM_NONFINITE) return RSFDE_E_NONFINITE;
      if (S.flag == GM_CONVERGED) {
        status = RSFDE_OK;
        break;
      }
    }
    CKS(run_cycle(h, I, mixed, u, &S, cyc));
    if (S.flag == GM_NONFINITE) return RSFDE_E_NONFINITE;
    st.iters += S.k;
    if (S.k > 0) {
      st.cycles += 1;
      I.k_prev[std::min(cyc, 2)] = S.k;
    }
    if (mixed) {
      // the cycle start just run found the FP64 residual below the bound
      if (S.k == 0 && S.flag == GM_CONVERGED) {
        status = RSFDE_OK;
        break;
      }
      st.outer_sweeps += 1;
    } else if (S.flag == GM_CONVERGED) {
      status = RSFDE_OK;
      break;
    }
    // a full cycle or a (near-)breakdown: the next cycle start recomputes the
    // residual and decides
  }
  if (mixed) {
    true_res = S.beta0 > 0 ? S.beta / S.beta0 : 0.0;
  } else if (h->true_res) {
    // recompute z = M (b - A u) in FP64 from the returned u (V_0 is free here)
    CKS(need_b());
    CKS(run_chain(h, I, CH_RESID, false, u, nullptr, I.b, 1.0, I.V));
    CK(kry_cycle_init(I.V, I.n, I.nb, I.st, I.partial, 0, p.rtol, inner_rtol, 0, p.restart, h->stream));
    GmresSummary R;
    CKS(read_summary(h, I, &R));
    if (!std::isfinite(R.beta)) return RSFDE_E_NONFINITE;
    true_res = R.beta0 > 0 ? R.beta / R.beta0 : 0.0;
  }
  if (stats) {
    stats->iters += st.iters;
    stats->cycles += st.cycles;
    stats->outer_sweeps += st.outer_sweeps;
    stats->converged = status == RSFDE_OK ? 1 : 0;
    stats->beta0 = S.beta0;
    stats->rel_pres = S.beta0 > 0 ? (mixed ? S.beta : S.res) / S.beta0 : 0.0;
    stats->rel_true_res = true_res;
  }
  return status;
}

// ---------------------------------------------------------------------------
// batched engine: all instances of a handle advance together.  Each pass
// position of a chain is one launch per group of instances sharing transform
// length, precision, axis kind and tile shape; each Krylov sweep, the update
// and the cycle start are one launch over all instances.  Instances keep their
// own GMRES state and stop on their own flags; the host drops an instance from
// the launches once its cycle has ended (its update applied exactly once).
// ---------------------------------------------------------------------------
static bool batchable(const rsfde_ctx* h) {
  if (h->count < 2) return false;
  const char* off = getenv("RSFDE_NO_BATCH");
  if (off && off[0] == '1') return false;
  // one chain shape and one restart length for all (the basis columns a launch
  // addresses exist in every instance)
  for (const Inst& I : h->inst)
    if (I.d != h->inst[0].d || I.p.precision != h->inst[0].p.precision ||
        I.p.restart != h->inst[0].p.restart || I.p.method != h->inst[0].p.method)
      return false;
  return true;
}

// Descriptor buffer capacity of one plan region for `count` instances: three
// chains of at most 12 pass positions (the two-sided operator chain in 3-D: its
// right factor, 5, and the operator with the left factor, 7) with a descriptor
// and a block-start entry per instance (64-byte aligned per group), the Krylov
// descriptors with two start arrays, and the source-operator jobs.
static size_t plan_capacity(int count) {
  const size_t per_pos = (size_t)count * (sizeof(BPass) + 3 * 64 + 8) + 64;
  return 3 * 12 * per_pos + (size_t)count * (sizeof(KBatch) + sizeof(FJob) + 32) + 8 * 64 + 4096;
}
static size_t fjob_capacity(int count) {
  return (size_t)count * (sizeof(FieldJob) + 8) + 4 * 64 + 1024;
}
static size_t batch_capacity(int count) {
  return 2 * plan_capacity(count) + fjob_capacity(count);
}

static void regions_init(rsfde_ctx* h) {
  const size_t pc = plan_capacity(h->count);
  h->rg[0] = {0, pc, 0};
  h->rg[1] = {pc, pc, 0};
  h->rg[2] = {2 * pc, fjob_capacity(h->count), 0};
}

// Append to region r's staging area; returns the device address of the copy
// (valid once the region is uploaded), or nullptr when the region is full.
static char* bappend(rsfde_ctx* h, int r, const void* src, size_t bytes) {
  rsfde_ctx::Region& R = h->rg[r];
  const size_t off = (R.fill + 63) & ~(size_t)63;
  if (off + bytes > R.cap) return nullptr;
  memcpy(h->bhost + R.base + off, src, bytes);
  R.fill = off + bytes;
  return h->bdev + R.base + off;
}

static hipError_t bupload(rsfde_ctx* h, int r) {
  const rsfde_ctx::Region& R = h->rg[r];
  if (R.fill == 0) return hipSuccess;
  return hipMemcpyAsync(h->bdev + R.base, h->bhost + R.base, R.fill, hipMemcpyHostToDevice, h->stream);
}

// Plan of one chain over the instance set S: record each instance's passes
// (same sequence of ops for every instance) and group them per position.
template <typename RecFn>
static int plan_chain(rsfde_ctx* h, int r, const std::vector<int>& S, RecFn rec_one, bool oper,
                      BChain& out) {
  std::vector<std::vector<RecPass>> recs(S.size());
  for (size_t s = 0; s < S.size(); ++s) {
    h->rec = &recs[s];
    h->rec_inst = S[s];
    const int st = rec_one(S[s]);
    h->rec = nullptr;
    if (st < 0) return st;
  }
  const size_t P = recs.empty() ? 0 : recs[0].size();
  for (auto& rc : recs)
    if (rc.size() != P) return RSFDE_E_STATE;
  out.pos.assign(P, {});
  for (size_t pi = 0; pi < P; ++pi) {
    std::vector<int> used(S.size(), 0);
    for (size_t s0 = 0; s0 < S.size(); ++s0) {
      if (used[s0]) continue;
      const RecPass& r0 = recs[s0][pi];
      const Inst& I0 = h->inst[r0.inst];
      BGroup g;
      g.L = I0.ax[r0.a.axis].L;
      g.var = r0.a.var;
      g.fp32 = r0.fp32;
      g.strided = r0.a.axis > 0;
      g.dht = r0.dht;
      if (g.dht) {
        // Hartley passes: grouped by length, axis kind and op
        g.op = r0.da.op;
        g.cls = g.op == DHT_SCALE ? RSFDE_K_DSD : RSFDE_K_DST;
        std::vector<DBPass> ddesc;
        std::vector<int> start(1, 0);
        for (size_t s = s0; s < S.size(); ++s) {
          const RecPass& rp = recs[s][pi];
          const Inst& I = h->inst[rp.inst];
          if (used[s] || !rp.dht || I.ax[rp.a.axis].L != g.L || (rp.a.axis > 0) != g.strided ||
              rp.da.op != g.op)
            continue;
          used[s] = 1;
          DBPass b;
          memset(&b, 0, sizeof(b));
          b.a = rp.da;
          b.ldv = I.ldv;
          if (oper) {
            if (rp.da.out == I.V + I.ldv) b.patch |= BP_OUT_J;
            if (rp.da.stop_fl == &I.st->FL[0]) b.patch |= BP_STOP;
          }
          ddesc.push_back(b);
          const int64_t nb = (rp.dnb + 7) / 8 * 8;
          if (start.back() + nb > 0x7fffffffLL) return RSFDE_E_UNSUPPORTED;
          start.push_back((int)(start.back() + nb));
          g.bytes += 16.0 * (double)I.n;
        }
        g.ninst = (int)ddesc.size();
        g.nblocks = start.back();
        g.ddesc = (const DBPass*)bappend(h, r, ddesc.data(), ddesc.size() * sizeof(DBPass));
        g.start = (const int*)bappend(h, r, start.data(), start.size() * sizeof(int));
        if (!g.ddesc || !g.start) return RSFDE_E_WORKSPACE;
        out.pos[pi].push_back(g);
        continue;
      }
      g.cls = op_class(r0.a.op);
      g.mv = r0.a.op <= OP_MV_LAST;
      std::vector<BPass> desc;
      std::vector<int> start(1, 0);
      for (size_t s = s0; s < S.size(); ++s) {
        const RecPass& rp = recs[s][pi];
        const Inst& I = h->inst[rp.inst];
        if (used[s] || rp.dht || I.ax[rp.a.axis].L != g.L || rp.a.var != g.var || rp.fp32 != g.fp32 ||
            (rp.a.axis > 0) != g.strided || rp.a.op != r0.a.op)
          continue;
        used[s] = 1;
        BPass b;
        memset(&b, 0, sizeof(b));
        b.a = rp.a;
        b.ldv = I.ldv;
        if (oper) {
          if (rp.a.in_c == (const void*)I.V) b.patch |= BP_IN_J;
          if (rp.a.out_a == (void*)(I.V + I.ldv)) b.patch |= BP_OUT_J;
          if (rp.a.use_gm) b.patch |= BP_GM;
          if (rp.stop_pend) b.patch |= BP_STOP_PEND;
          else if (rp.a.stop_fl == &I.st->FL[0]) b.patch |= BP_STOP;
        }
        desc.push_back(b);
        const int64_t nb = (rp.a.nlaunch + 7) / 8 * 8;  // 8-aligned: XCD order kept per instance
        if (start.back() + nb > 0x7fffffffLL) return RSFDE_E_UNSUPPORTED;
        start.push_back((int)(start.back() + nb));
        g.bytes += pass_bytes(rp.a, I, rp.fp32);
      }
      g.ninst = (int)desc.size();
      g.nblocks = start.back();
      g.desc = (const BPass*)bappend(h, r, desc.data(), desc.size() * sizeof(BPass));
      g.start = (const int*)bappend(h, r, start.data(), start.size() * sizeof(int));
      if (!g.desc || !g.start) return RSFDE_E_WORKSPACE;
      out.pos[pi].push_back(g);
    }
  }
  return RSFDE_OK;
}

static int launch_chain_batched(rsfde_ctx* h, const BChain& c, int j, int pend) {
  for (const auto& pos : c.pos)
    for (const BGroup& g : pos) {
      if (g.nblocks <= 0) continue;
      if (g.dht) {
        DBLaunch dl;
        dl.desc = g.ddesc;
        dl.start = g.start;
        dl.ninst = g.ninst;
        dl.j = j;
        CKS(timed_launch(h, g.cls, g.bytes, [&](hipEvent_t ea, hipEvent_t eb) -> hipError_t {
          if (ea) {
            hipError_t e = hipEventRecord(ea, h->stream);
            if (e != hipSuccess) return e;
          }
          hipError_t e = launch_dht_batched(g.L, dl, g.nblocks, g.strided, h->stream);
          if (e == hipSuccess && eb) e = hipEventRecord(eb, h->stream);
          return e;
        }));
        continue;
      }
      BLaunch bl;
      bl.desc = g.desc;
      bl.start = g.start;
      bl.ninst = g.ninst;
      bl.j = j;
      bl.pend = pend;
      bl.mv = g.mv ? 1 : 0;
      CKS(timed_launch(h, g.cls, g.bytes, [&](hipEvent_t ea, hipEvent_t eb) {
        return launch_pass_batched(g.L, g.fp32, bl, g.nblocks, g.strided, g.var, h->stream, ea, eb);
      }));
    }
  return RSFDE_OK;
}


static int plan_krylov(rsfde_ctx* h, int r, const std::vector<int>& S, double* const* u, KPlan& kp) {
  std::vector<KBatch> desc;
  std::vector<int> snb(1, 0), snbu(1, 0);
  kp = KPlan();
  for (int i : S) {
    Inst& I = h->inst[i];
    KBatch d;
    memset(&d, 0, sizeof(d));
    d.k.V = I.V;
    d.k.ldv = I.ldv;
    d.k.n = I.n;
    d.k.w = I.V + I.ldv;
    d.k.st = I.st;
    d.k.pa = I.pk[0];
    d.k.pb = I.pk[1];
    d.k.pc = I.pk[2];
    d.k.j = 0;
    d.k.m = I.p.restart;
    // two-sided form: the update writes V y to T[3]; the host adds P^{-1/2} of it to u
    const bool two = I.p.method == RSFDE_TPGM;
    d.x = two ? (double*)I.tmp[3] : u[i];
    d.overwrite = two ? 1 : 0;
    d.partial = I.partial;
    d.rtol = I.p.precision == RSFDE_MIXED ? outer_tol(I.p) : I.p.rtol;
    d.inner_rtol = inner_tol(I.p);
    d.k.nb = I.nb;
    d.nb = I.nb;
    d.nbu = upd_blocks(I.n);
    d.mixed = I.p.precision == RSFDE_MIXED ? 1 : 0;
    desc.push_back(d);
    snb.push_back(snb.back() + d.nb);
    snbu.push_back(snbu.back() + d.nbu);
    kp.vbytes += 8.0 * (double)I.n;
    kp.m = std::max(kp.m, I.p.restart);
  }
  kp.ninst = (int)S.size();
  kp.nb_total = snb.back();
  kp.nbu_total = snbu.back();
  kp.desc = (const KBatch*)bappend(h, r, desc.data(), desc.size() * sizeof(KBatch));
  kp.start_nb = (const int*)bappend(h, r, snb.data(), snb.size() * sizeof(int));
  kp.start_nbu = (const int*)bappend(h, r, snbu.data(), snbu.size() * sizeof(int));
  if (!kp.desc || !kp.start_nb || !kp.start_nbu) return RSFDE_E_WORKSPACE;
  return RSFDE_OK;
}

static KLaunch klaunch(const KPlan& kp, bool upd, int j, int pend, int first, const int* mask) {
  KLaunch kl;
  kl.desc = kp.desc;
  kl.start = upd ? kp.start_nbu : kp.start_nb;
  kl.ninst = kp.ninst;
  kl.j = j;
  kl.pend = pend;
  kl.first = first;
  kl.mask = mask;
  return kl;
}

// Plans for the set S in region r: the source-operator jobs and the
// right-hand side chain (when prep), the residual and operator chains and the
// Krylov descriptors; uploaded in one copy.

static int build_plans(rsfde_ctx* h, int r, const std::vector<int>& S, double* const* u,
                       const double* const* f_half, bool prep, bool fp32, BPlan& bp) {
  CK(hipStreamSynchronize(h->stream));  // earlier copies out of the staging area are done
  h->rg[r].fill = 0;
  bp = BPlan();
  if (prep) {
    std::vector<FJob> jobs;
    std::vector<int> start(1, 0);
    for (int i : S) {
      Inst& I = h->inst[i];
      FJob J;
      memset(&J, 0, sizeof(J));
      J.fcl = f_half[i];
      J.g = grid_dev(I, false);
      for (int a = 0; a < 3; ++a) J.al[a] = I.p.alpha[a];
      J.F = I.F;
      jobs.push_back(J);
      start.push_back(start.back() + (int)((I.n + 255) / 256));
    }
    bp.nf = (int)jobs.size();
    bp.fblocks = start.back();
    bp.fjobs = (const FJob*)bappend(h, r, jobs.data(), jobs.size() * sizeof(FJob));
    bp.fstart = (const int*)bappend(h, r, start.data(), start.size() * sizeof(int));
    if (!bp.fjobs || !bp.fstart) return RSFDE_E_WORKSPACE;
    CKS(plan_chain(h, r, S, [&](int i) {
      Inst& I = h->inst[i];
      return run_chain(h, I, CH_RHS, false, u[i], nullptr, I.F, I.p.dt, I.b);
    }, false, bp.rhs));
  }
  CKS(plan_chain(h, r, S, [&](int i) {
    Inst& I = h->inst[i];
    return run_chain(h, I, CH_RESID, false, u[i], nullptr, I.b, 1.0, I.V);
  }, false, bp.resid));
  CKS(plan_chain(h, r, S, [&](int i) {
    Inst& I = h->inst[i];
    GmRes g;
    g.st = I.st;
    g.p3 = I.pk[2];
    g.nb3 = I.nb;
    g.j = 0;
    g.pend = -1;
    g.m = I.p.restart;
    return run_chain(h, I, CH_OPER, fp32, I.V, nullptr, nullptr, 0.0, I.V + I.ldv, &g, &I.st->FL[0]);
  }, true, bp.oper));
  CKS(plan_krylov(h, r, S, u, bp.kp));
  CK(bupload(h, r));
  return RSFDE_OK;
}

static int read_summaries(rsfde_ctx* h, const KPlan& kp) {
  CK(kry_gather_summaries(kp.desc, kp.ninst, h->dsum, h->stream));
  CK(hipMemcpyAsync(h->psum, h->dsum, kp.ninst * sizeof(GmresSummary), hipMemcpyDeviceToHost,
                    h->stream));
  CK(stream_wait(h));
  if (!h->pending.empty()) {
    // a batched launch of step j did work while some instance's cycle had not
    // ended before j (instances that ended earlier exit inside it)
    int kend = 0;
    for (int s = 0; s < kp.ninst; ++s)
      kend = std::max(kend, h->psum[s].flag == GM_RUNNING ? RSFDE_MAX_RESTART + 1 : h->psum[s].k);
    mark_speculative(h, kend);
    CKS(flush_timing(h));
  }
  return RSFDE_OK;
}

// One lockstep GMRES cycle over the plan's instance set (cycle start already
// launched); on return fin[i] holds each instance's final summary of the cycle.
// An instance whose cycle ended in an earlier chunk stays in the launches (its
// kernels exit on its status words) but its update is masked off, so V y is
// added exactly once.
static int run_cycle_batched(rsfde_ctx* h, const std::vector<int>& S, bool fp32, BPlan& bp,
                             std::vector<GmresSummary>& fin, int cyc) {
  (void)fp32;
  int kprev = 1;
  for (int i : S) kprev = std::max(kprev, h->inst[i].k_prev[std::min(cyc, 2)]);
  const int ns = (int)S.size();
  for (int s = 0; s < ns; ++s) h->pmask[s] = 1;
  CK(hipMemcpyAsync(h->dmask, h->pmask, ns * sizeof(int), hipMemcpyHostToDevice, h->stream));
  std::vector<char> done(ns, 0);
  int j = 0, pending = -1;
  int chunk = std::max(1, std::min(bp.kp.m, kprev));
  while (true) {
    const int m = bp.kp.m;
    const int jend = std::min(m, j + chunk);
    for (int jj = j; jj < jend; ++jj) {
      const int pend = jj == j ? pending : jj - 1;
      auto launch = [&]() -> int {
        h->cur_step = jj;
        CKS(launch_chain_batched(h, bp.oper, jj, pend));
        for (int w = 1; w <= 2; ++w) {
          const KLaunch kl = klaunch(bp.kp, false, jj, -1, 0, nullptr);
          const int cls = w == 1 ? RSFDE_K_DOTS : RSFDE_K_ORTH_DOTS;
          const int words = w == 1 ? jj + 2 : jj + 2 + (jj >= 1 ? 2 : 1);
          CKS(timed_launch(h, cls, bp.kp.vbytes * words, [&](hipEvent_t ea, hipEvent_t eb) {
            return kry_sweep_batched(w, kl, bp.kp.nb_total, h->stream, ea, eb);
          }));
        }
        h->cur_step = -1;
        return RSFDE_OK;
      };
      if (h->graphs && h->tmask == 0 && &bp == &h->full) {
        if (h->bg_gen != h->plan_gen) {
          graphs_clear(h->bgexec);
          h->bg_gen = h->plan_gen;
        }
        CKS(graph_step(h, h->bgexec, (size_t)(2 * jj + (pend >= 0 ? 1 : 0)), launch));
      } else {
        CKS(launch());
      }
    }
    const KLaunch ku = klaunch(bp.kp, true, jend - 1, jend - 1, 0, h->dmask);
    CKS(timed_launch(h, RSFDE_K_UPDATE, 0.0, [&](hipEvent_t ea, hipEvent_t eb) {
      return kry_update_batched(ku, bp.kp.nbu_total, h->stream, ea, eb);
    }));
    CKS(read_summaries(h, bp.kp));
    int running = 0, need = 1;
    bool newly = false;
    for (int s = 0; s < ns; ++s) {
      if (done[s]) continue;
      const GmresSummary& G = h->psum[s];
      if (G.flag == GM_RUNNING) {
        ++running;
        need = std::max(need, next_chunk(G, jend, bp.kp.m - jend));
      } else {
        fin[S[s]] = G;
        done[s] = 1;
        h->pmask[s] = 0;
        newly = true;
      }
    }
    if (running == 0) return RSFDE_OK;
    j = jend;
    pending = -1;
    chunk = need;
    if (j >= bp.kp.m) return RSFDE_OK;  // cannot happen: the last step of a cycle never runs on
    if (newly) CK(hipMemcpyAsync(h->dmask, h->pmask, ns * sizeof(int), hipMemcpyHostToDevice, h->stream));
  }
}

static int step_batched(rsfde_ctx* h, const double* const* e_half, const double* const* f_half,
                        double* const* u, rsfde_stats* stats) {
  const int C = h->count;
  const bool mixed = h->inst[0].p.precision == RSFDE_MIXED;
  for (int i = 0; i < C; ++i) {
    Inst& I = h->inst[i];
    if (!I.ebar_set) return RSFDE_E_STATE;
    if ((uintptr_t)u[i] & 15) return RSFDE_E_INVALID_ARG;
    I.ecur = e_half[i];  // read in place
  }
  std::vector<int> act(C);
  for (int i = 0; i < C; ++i) act[i] = i;
  // the full-set plan is reused while the step's buffers repeat
  std::vector<const void*> key(3 * C);
  for (int i = 0; i < C; ++i) {
    key[3 * i] = u[i];
    key[3 * i + 1] = e_half[i];
    key[3 * i + 2] = f_half[i];
  }
  if (!h->full_valid || key != h->full_key) {
    h->full_valid = false;
    CKS(build_plans(h, 0, act, u, f_half, true, mixed, h->full));
    h->full_key = key;
    h->full_valid = true;
    ++h->plan_gen;  // graphs captured on the previous plan are stale
  }
  BPlan& bp0 = h->full;
  CK(compute_F_batched(bp0.fjobs, bp0.fstart, bp0.nf, bp0.fblocks, h->stream));
  if (mixed)
    for (int i = 0; i < C; ++i) CK(convert_f64_f32(h->inst[i].ecur, h->inst[i].e32, h->inst[i].n, h->stream));
  CKS(launch_chain_batched(h, bp0.rhs, 0, -1));
  for (int i = 0; i < C; ++i)
    if (h->inst[i].p.x0_mode == 1) CK(fill_f64(u[i], h->inst[i].n, 0.0, h->stream));
  std::vector<int> status(C, RSFDE_W_NOT_CONVERGED);
  std::vector<rsfde_stats> st(C);
  memset(st.data(), 0, sizeof(rsfde_stats) * C);
  std::vector<GmresSummary> last(C);
  memset(last.data(), 0, sizeof(GmresSummary) * C);
  BPlan sub;
  for (int cyc = 0; !act.empty(); ++cyc) {
    BPlan* bp = &bp0;
    if ((int)act.size() < C) {
      CKS(build_plans(h, 1, act, u, f_half, false, mixed, sub));
      bp = &sub;
    }
    CKS(launch_chain_batched(h, bp->resid, 0, -1));
    {
      const KLaunch kl = klaunch(bp->kp, false, 0, -1, cyc == 0 ? 1 : 0, nullptr);
      CK(kry_norm_batched(kl, bp->kp.nb_total, h->stream));
      CK(kry_cycle_fin_batched(kl, h->stream));
    }
    std::vector<int> go;  // instances that run a cycle now
    if (mixed) {
      // instances at their last outer sweep only check the refined residual; a
      // refinement sweep's start (cyc >= 1) usually finds it below the bound
      // already, so the starts are read before any steps are launched
      bool any_final = false;
      for (int i : act) {
        const int max_outer = h->inst[i].p.max_outer > 0 ? h->inst[i].p.max_outer : 30;
        if (cyc == max_outer) any_final = true;
      }
      if (any_final || cyc > 0) {
        CKS(read_summaries(h, bp->kp));
        for (size_t s = 0; s < act.size(); ++s) {
          const int i = act[s];
          const int max_outer = h->inst[i].p.max_outer > 0 ? h->inst[i].p.max_outer : 30;
          const GmresSummary& G = h->psum[s];
          if (G.flag == GM_NONFINITE) return RSFDE_E_NONFINITE;
          if (cyc == max_outer) {
            last[i] = G;
            if (G.flag == GM_CONVERGED) status[i] = RSFDE_OK;
          } else if (G.flag == GM_CONVERGED) {
            last[i] = G;
            status[i] = RSFDE_OK;
          } else {
            go.push_back(i);
          }
        }
        if (!go.empty() && go.size() < act.size()) {
          CKS(build_plans(h, 1, go, u, f_half, false, mixed, sub));
          bp = &sub;
        }
      } else {
        go = act;
      }
    } else {
      go = act;
    }
    if (go.empty()) break;
    std::vector<GmresSummary> fin(C);
    memset(fin.data(), 0, sizeof(GmresSummary) * C);
    CKS(run_cycle_batched(h, go, mixed, *bp, fin, cyc));
    if (h->inst[0].p.method == RSFDE_TPGM) {
      // u += P^{-1/2} (V y) for the instances whose cycle ended with an update: one
      // batched chain of the right factor whose last pass adds into u (plan region 1
      // is free when the cycle ran the full-set plan; else appended after its plan)
      std::vector<int> corr;
      for (int i : go)
        if (fin[i].flag != GM_NONFINITE && fin[i].k > 0) corr.push_back(i);
      if (!corr.empty()) {
        if (bp == &bp0) h->rg[1].fill = 0;
        BChain cc;
        CKS(plan_chain(h, 1, corr, [&](int i) {
          Inst& I = h->inst[i];
          return run_prec(h, I, false, (const double*)I.tmp[3], u[i], PM_PH, nullptr, nullptr, true);
        }, false, cc));
        CK(bupload(h, 1));
        CKS(launch_chain_batched(h, cc, 0, -1));
      }
    }
    std::vector<int> next;
    for (int i : go) {
      Inst& I = h->inst[i];
      const GmresSummary& S = fin[i];
      last[i] = S;
      if (S.flag == GM_NONFINITE) return RSFDE_E_NONFINITE;
      st[i].iters += S.k;
      if (S.k > 0) {
        st[i].cycles += 1;
        I.k_prev[std::min(cyc, 2)] = S.k;
      }
      bool done = false;
      if (mixed) {
        if (S.k == 0 && S.flag == GM_CONVERGED) {
          status[i] = RSFDE_OK;
          done = true;
        } else {
          st[i].outer_sweeps += 1;
        }
      } else {
        // a full cycle or a (near-)breakdown starts a new cycle, whose start
        // recomputes the residual and decides
        if (S.flag == GM_CONVERGED) {
          status[i] = RSFDE_OK;
          done = true;
        } else if (cyc + 1 >= I.p.max_cycles) {
          done = true;
        }
      }
      if (!done) next.push_back(i);
    }
    act = next;
  }
  std::vector<double> true_res(C, -1.0);
  for (int i = 0; i < C; ++i) {
    if (mixed) {
      true_res[i] = last[i].beta0 > 0 ? last[i].beta / last[i].beta0 : 0.0;
    } else if (h->true_res) {
      // the recomputed FP64 residual of each instance, one at a time (V_0 is free)
      Inst& I = h->inst[i];
      CKS(run_chain(h, I, CH_RESID, false, u[i], nullptr, I.b, 1.0, I.V));
      CK(kry_cycle_init(I.V, I.n, I.nb, I.st, I.partial, 0, I.p.rtol, inner_tol(I.p), 0, I.p.restart,
                        h->stream));
      GmresSummary R;
      CKS(read_summary(h, I, &R));
      if (!std::isfinite(R.beta)) return RSFDE_E_NONFINITE;
      true_res[i] = R.beta0 > 0 ? R.beta / R.beta0 : 0.0;
    }
  }
  int worst = RSFDE_OK;
  for (int i = 0; i < C; ++i) {
    if (stats) {
      rsfde_stats& o = stats[i];
      o.iters += st[i].iters;
      o.cycles += st[i].cycles;
      o.outer_sweeps += st[i].outer_sweeps;
      o.converged = status[i] == RSFDE_OK ? 1 : 0;
      o.beta0 = last[i].beta0;
      o.rel_pres = last[i].beta0 > 0 ? (mixed ? last[i].beta : last[i].res) / last[i].beta0 : 0.0;
      o.rel_true_res = true_res[i];
    }
    worst = std::max(worst, status[i]);
  }
  return worst;
}

// ---------------------------------------------------------------------------
// tile and radix-plan autotuner: time the variants of every pass kind the chains
// use (operator pass and transform pass, per axis and precision) on the
// instance's own grid and keep the fastest.  Variants 0 .. 2 change only how many
// pencils a workgroup holds (bitwise the same results); variants 3 .. 5 run the
// length's alternative radix plan (the same transform, rounded differently).
// Choices are kept per device architecture in a process-wide cache keyed by
// (dimension, axis, precision, pass kind, length), so that every handle of the
// process -- one instance or many -- runs the same kernels for the same pass and
// batched and one-at-a-time runs stay bit-identical.  The cache starts from
// tune_cache.txt beside the library (read only), or from RSFDE_TUNE_CACHE=<file>,
// which also receives the new choices (one key=variant line each).  RSFDE_NO_AUTOTUNE=1 keeps variant 0;
// RSFDE_FORCE_VARIANT=v runs variant v wherever the length has it (tests).
// ---------------------------------------------------------------------------
namespace {
std::mutex g_tune_mu;
std::vector<std::pair<std::string, int>> g_tune;  // key -> variant
bool g_tune_loaded = false;
}  // namespace

static std::string tune_key(const char* arch, int d, int ax, int fp, int cls, int L) {
  char b[160];
  snprintf(b, sizeof b, "%s d%d ax%d fp%d cls%d L%d", arch, d, ax, fp, cls, L);
  return b;
}

// Cache file read when RSFDE_TUNE_CACHE is not set: tune_cache.txt beside the
// library (the choices shipped with it; read only).
static std::string default_tune_cache() {
  Dl_info info;
  if (dladdr((void*)&default_tune_cache, &info) && info.dli_fname) {
    std::string p = info.dli_fname;
    const size_t slash = p.rfind('/');
    return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/tune_cache.txt";
  }
  return std::string();
}

// Looks the key up (loading the cache file once); -1 when absent.
static int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_loaded) {
    g_tune_loaded = true;
    const char* env = getenv("RSFDE_TUNE_CACHE");
    const std::string path = env && env[0] ? std::string(env) : default_tune_cache();
    if (!path.empty()) {
      FILE* fh = fopen(path.c_str(), "r");
      if (fh) {
        char line[256];
        while (fgets(line, sizeof line, fh)) {
          char* eq = strrchr(line, '=');
          if (!eq) continue;
          *eq = 0;
          const int v = atoi(eq + 1);
          if (v >= 0 && v < RSFDE_PASS_VARIANTS) g_tune.emplace_back(line, v);
        }
        fclose(fh);
      }
    }
  }
  for (const auto& e : g_tune)
    if (e.first == key) return e.second;
  return -1;
}

static void tune_store(const std::string& key, int v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.emplace_back(key, v);
  const char* path = getenv("RSFDE_TUNE_CACHE");
  if (path && path[0]) {
    FILE* fh = fopen(path, "a");
    if (fh) {
      fprintf(fh, "%s=%d\n", key.c_str(), v);
      fclose(fh);
    }
  }
}

static int autotune(rsfde_ctx* h, Inst& I) {
  const char* off = getenv("RSFDE_NO_AUTOTUNE");
  if (off && off[0] == '1') return RSFDE_OK;
  const char* fv = getenv("RSFDE_FORCE_VARIANT");
  const int forced = fv && fv[0] ? atoi(fv) : -1;
  const char* vb = getenv("RSFDE_AUTOTUNE_VERBOSE");
  const bool verbose = vb && vb[0] == '1';
  const int nprec = I.p.precision == RSFDE_MIXED ? 2 : 1;
  const int d = I.d;
  if (forced >= 0) {
    for (int ax = 0; ax < d; ++ax)
      for (int fp = 0; fp < nprec; ++fp)
        for (int cls = 0; cls < 2; ++cls) {
          int nt = 0, ppt = 0;
          pass_shape_rt(I.ax[ax].L, fp == 1, ax > 0, forced, &nt, &ppt);
          I.var[ax][fp][cls] = nt > 0 ? forced : 0;
        }
    return RSFDE_OK;
  }
  char arch[64] = "gfx";
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      strncpy(arch, prop.gcnArchName, sizeof arch - 1);
      arch[sizeof arch - 1] = 0;
      for (char* c = arch; *c; ++c)
        if (*c == ' ' || *c == '=') *c = '_';
    }
  }
  for (int k = 0; k < 4; ++k) CK(fill_f64((double*)I.tmp[k], I.n, 0.0, h->stream));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  int status = RSFDE_OK;
  for (int ax = 0; ax < d && status == RSFDE_OK; ++ax) {
    for (int fp = 0; fp < nprec && status == RSFDE_OK; ++fp) {
      for (int cls = 0; cls < 2 && status == RSFDE_OK; ++cls) {
        if (cls == 1 && d == 1) continue;  // one-axis chains have no transform pass
        int op, flags = 0;
        if (cls == 1) {
          op = ax == 0 ? OP_DSD : OP_DST;
        } else if (d == 1) {
          op = OP_MV_LAST;
          flags = FL_FIRST_IS_LAST | FL_IN64 | FL_OUT64 | FL_PREC_FULL;
        } else if (ax == 0) {
          op = OP_MV_FIRST;
          flags = FL_IN64;
        } else if (ax < d - 1) {
          op = OP_MV_MID;
        } else {
          op = OP_MV_LAST;
          flags = FL_DST_AFTER;
        }
        const int L = I.ax[ax].L;
        const std::string key = tune_key(arch, d, ax, fp, cls, L);
        const int cached = tune_lookup(key);
        if (cached >= 0) {
          int nt = 0, ppt = 0;
          pass_shape_rt(L, fp == 1, ax > 0, cached, &nt, &ppt);
          if (nt > 0) {
            I.var[ax][fp][cls] = cached;
            continue;
          }
        }
        // variants interleaved over five rounds, each timing four launches whose
        // inputs and outputs rotate over the four temporaries (inputs are not
        // left cache-resident by the previous launch); the best round counts
        float tbest[RSFDE_PASS_VARIANTS];
        bool have[RSFDE_PASS_VARIANTS];
        for (int v = 0; v < RSFDE_PASS_VARIANTS; ++v) {
          int nt = 0, ppt = 0;
          pass_shape_rt(L, fp == 1, ax > 0, v, &nt, &ppt);
          have[v] = nt > 0;
          tbest[v] = 1e30f;
        }
        for (int rep = 0; rep < 5 && status == RSFDE_OK; ++rep) {
          for (int v = 0; v < RSFDE_PASS_VARIANTS && status == RSFDE_OK; ++v) {
            if (!have[v]) continue;
            I.var[ax][fp][cls] = v;
            PassArgs t = mk_pass(I, ax, op, fp == 1);
            t.flags = flags;
            hipError_t e = hipEventRecord(e0, h->stream);
            for (int r = 0; r < 4 && e == hipSuccess; ++r) {
              const int k = rep + r + v;
              t.in_c = I.tmp[k & 3];
              t.in_a = I.tmp[(k + 1) & 3];
              t.out_a = I.tmp[(k + 2) & 3];
              t.out_c = I.tmp[(k + 3) & 3];
              e = launch_pass(L, fp == 1, t, ax > 0, h->stream);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
              g_last_hip = e;
              status = RSFDE_E_HIP;
              break;
            }
            if (ms < tbest[v]) tbest[v] = ms;
          }
        }
        // the default plan's widest tile unless another tile is 3 % faster or the
        // alternative plan 5 % faster (a plan change moves the rounding as well)
        int bestv = 0;
        for (int v = 1; v < RSFDE_PASS_VARIANTS; ++v)
          if (have[v] && tbest[v] < tbest[bestv] * (v >= 3 && bestv < 3 ? 0.95f : 0.97f)) bestv = v;
        if (verbose) {
          fprintf(stderr, "rsfde autotune: %s axis %d %s %s pass, L %d:", arch, ax,
                  fp ? "fp32" : "fp64", cls ? "transform" : "operator", L);
          for (int v = 0; v < RSFDE_PASS_VARIANTS; ++v)
            if (have[v]) fprintf(stderr, " v%d %.1f", v, 250.f * tbest[v]);
          fprintf(stderr, " us per launch -> variant %d\n", bestv);
        }
        I.var[ax][fp][cls] = bestv;
        if (status == RSFDE_OK) tune_store(key, bestv);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int rsfde_workspace_size(const rsfde_params* p, int count, size_t* bytes) {
  if (!p || !bytes || count < 1) return RSFDE_E_INVALID_ARG;
  Bump B{nullptr};
  for (int i = 0; i < count; ++i) {
    const int v = validate(&p[i]);
    if (v != RSFDE_OK) return v;
    Inst I;
    I.p = p[i];
    layout(I, B);
  }
  if (count > 1) {
    (void)B.take<char>(batch_capacity(count));
    (void)B.take<GmresSummary>((size_t)count);
    (void)B.take<int>((size_t)count);
  }
  *bytes = (B.off + 255) & ~(size_t)255;
  return RSFDE_OK;
}

int rsfde_setup(const rsfde_params* p, int count, void* workspace, size_t bytes, void* stream,
                rsfde_handle* out) {
  if (!p || !out || count < 1) return RSFDE_E_INVALID_ARG;
  size_t need = 0;
  const int v = rsfde_workspace_size(p, count, &need);
  if (v != RSFDE_OK) return v;
  if (!workspace || bytes < need || ((uintptr_t)workspace & 255)) return RSFDE_E_WORKSPACE;
  {
    // the no-allocation entry point's device scratch: take its address on this
    // device now (set-up), so the entry point itself only looks it up
    void* sp = nullptr;
    CK(scratch_ptr(&sp));
  }
  rsfde_ctx* h = new (std::nothrow) rsfde_ctx();
  if (!h) return RSFDE_E_INVALID_ARG;
  h->count = count;
  h->stream = (hipStream_t)stream;
  h->inst.resize(count);
  Bump B{(char*)workspace};
  int status = RSFDE_OK;
  hipError_t he = hipHostMalloc((void**)&h->pinned, sizeof(GmresSummary), hipHostMallocDefault);
  if (he == hipSuccess && count > 1) {
    h->bcap = batch_capacity(count);
    he = hipHostMalloc((void**)&h->bhost, h->bcap, hipHostMallocDefault);
    if (he == hipSuccess)
      he = hipHostMalloc((void**)&h->psum, (size_t)count * sizeof(GmresSummary), hipHostMallocDefault);
    if (he == hipSuccess) he = hipHostMalloc((void**)&h->pmask, (size_t)count * sizeof(int), hipHostMallocDefault);
  }
  if (he != hipSuccess) {
    g_last_hip = he;
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->bhost) (void)hipHostFree(h->bhost);
    if (h->psum) (void)hipHostFree(h->psum);
    delete h;
    return RSFDE_E_HIP;
  }
  for (int i = 0; i < count && status == RSFDE_OK; ++i) {
    Inst& I = h->inst[i];
    I.p = p[i];
    layout(I, B);
    I.nb = count > 1 ? kry_blocks_many(I.n) : kry_blocks(I.n);
    double pscale = 1.0;
    int64_t inner = 1;
    for (int a = 0; a < I.d; ++a) {
      Axis& A = I.ax[a];
      A.alpha = p[i].alpha[a];
      A.h = (p[i].hi[a] - p[i].lo[a]) / (double)(A.N + 1);
      A.eta = p[i].kappa[a] * p[i].dt / (2.0 * pow(A.h, A.alpha));
      A.inner = inner;
      inner *= A.N;
      pscale /= (double)A.L;
      hipError_t e = setup_axis_tables(A.alpha, A.N, A.L, A.eta, A.s, A.tw64, A.tw32, A.chat64,
                                       A.chat32, A.q, A.lam64, A.lam32, A.wq64, A.wq32, h->stream);
      if (e == hipSuccess && I.p.method == RSFDE_SPGM)
        e = setup_strang_tables(A.L, A.alpha, A.N, A.eta, A.s, A.tw64, A.chirp, A.khat, A.slam,
                                A.swq, h->stream);
      if (e != hipSuccess) {
        g_last_hip = e;
        status = RSFDE_E_HIP;
        break;
      }
    }
    I.pscale = pscale;
    if (status != RSFDE_OK) break;
    if (kry_state_reset(I.st, h->stream) != hipSuccess ||
        hipMemsetAsync(I.counters, 0, 64 * sizeof(unsigned), h->stream) != hipSuccess) {
      g_last_hip = hipGetLastError();
      status = RSFDE_E_HIP;
      break;
    }
    if (!(p[i].e_min == 0.0 && p[i].e_max == 0.0)) {
      const double eb = 0.5 * (p[i].e_min + p[i].e_max);
      I.ebar_h = eb;
      I.ebar_set = true;
      if (hipMemcpyAsync(I.ebar, &I.ebar_h, sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
        status = RSFDE_E_HIP;
        break;
      }
    }
  }
  if (status == RSFDE_OK && count > 1) {
    h->bdev = B.take<char>(h->bcap);
    h->dsum = B.take<GmresSummary>((size_t)count);
    h->dmask = B.take<int>((size_t)count);
    regions_init(h);
    h->batched = batchable(h);
  }
  if (status == RSFDE_OK) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      g_last_hip = e;
      status = RSFDE_E_HIP;
    }
  }
  for (int i = 0; i < count && status == RSFDE_OK; ++i) status = autotune(h, h->inst[i]);
  if (status != RSFDE_OK) {
    (void)hipHostFree(h->pinned);
    if (h->bhost) (void)hipHostFree(h->bhost);
    if (h->psum) (void)hipHostFree(h->psum);
    if (h->pmask) (void)hipHostFree(h->pmask);
    delete h;
    return status;
  }
  *out = h;
  return RSFDE_OK;
}

int rsfde_set_ebar(rsfde_handle h, int instance, double e_min, double e_max) {
  if (!h || instance < 0 || instance >= h->count) return RSFDE_E_INVALID_ARG;
  if (!(e_min > 0.0 && e_min <= e_max && isfinite(e_max))) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  I.ebar_h = 0.5 * (e_min + e_max);
  CK(hipMemcpyAsync(I.ebar, &I.ebar_h, sizeof(double), hipMemcpyHostToDevice, h->stream));
  CK(hipStreamSynchronize(h->stream));
  I.ebar_set = true;
  return RSFDE_OK;
}

int rsfde_step(rsfde_handle h, double t_m, const double* const* e_half, const double* const* f_half,
               double* const* u, rsfde_stats* stats) {
  (void)t_m;
  if (!h || !e_half || !f_half || !u) return RSFDE_E_INVALID_ARG;
  for (int i = 0; i < h->count; ++i)
    if (!e_half[i] || !f_half[i] || !u[i]) return RSFDE_E_INVALID_ARG;
  int worst = RSFDE_OK;
  if (stats) memset(stats, 0, sizeof(rsfde_stats) * h->count);
  if (h->batched) {
    worst = step_batched(h, e_half, f_half, u, stats);
    if (worst < 0) return worst;
  } else {
    for (int i = 0; i < h->count; ++i) {
      const int s = step_one(h, h->inst[i], e_half[i], f_half[i], u[i], stats ? &stats[i] : nullptr);
      if (s < 0) return s;
      if (s > worst) worst = s;
    }
  }
  CK(hipStreamSynchronize(h->stream));
  return worst;
}

static int builtin_sample(rsfde_ctx* h, Inst& I, double t, bool need_f) {
  if (!(I.fe.set && !I.fe.spec.time_dependent && I.fe.evaluated)) {
    CKS(eval_field(h, I, RSFDE_WHICH_E, t, I.e));
    if (!I.fe.spec.time_dependent) I.fe.evaluated = true;
  }
  if (need_f && !(I.ff.set && !I.ff.spec.time_dependent && I.ff.evaluated)) {
    CKS(eval_field(h, I, RSFDE_WHICH_F, t, I.f));
    if (!I.ff.spec.time_dependent) I.ff.evaluated = true;
  }
  return RSFDE_OK;
}

int rsfde_solve(rsfde_handle h, int M, rsfde_sample_fn sample, void* ctx, double* const* u,
                rsfde_stats* stats) {
  return rsfde_solve_range(h, 0, M, sample, ctx, u, stats);
}

int rsfde_solve_range(rsfde_handle h, int m0, int M, rsfde_sample_fn sample, void* ctx,
                      double* const* u, rsfde_stats* stats) {
  if (!h || m0 < 0 || M < 0 || !u) return RSFDE_E_INVALID_ARG;
  for (int i = 0; i < h->count; ++i) {
    if (!u[i]) return RSFDE_E_INVALID_ARG;
    if (!sample && !h->inst[i].fe.set) return RSFDE_E_STATE;
  }
  if (stats) memset(stats, 0, sizeof(rsfde_stats) * h->count);
  // ebar pre-scan over all midpoints (eq. dhat) where it is not known yet
  for (int i = 0; i < h->count; ++i) {
    Inst& I = h->inst[i];
    if (I.ebar_set) continue;
    CK(minmax_reset(I.eminmax, h->stream));
    const bool tindep = !sample && !I.fe.spec.time_dependent;
    const int scans = tindep ? std::min(M, 1) : M;
    for (int m = 0; m < scans; ++m) {
      const double th = (m0 + m + 0.5) * I.p.dt;
      if (sample) {
        if (sample(ctx, i, th, I.e, I.f, (void*)h->stream) != 0) return RSFDE_E_INVALID_ARG;
      } else {
        CKS(eval_field(h, I, RSFDE_WHICH_E, th, I.e));
      }
      CK(minmax_accum(I.e, I.n, I.eminmax, I.partial, I.counters + 2, h->stream));
    }
    double mm[2];
    CK(hipMemcpyAsync(mm, I.eminmax, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    CK(hipStreamSynchronize(h->stream));
    if (!(mm[0] > 0.0) || !isfinite(mm[1])) return RSFDE_E_INVALID_ARG;
    CKS(rsfde_set_ebar(h, i, mm[0], mm[1]));
  }
  int worst = RSFDE_OK;
  std::vector<const double*> ep(h->count), fp(h->count);
  std::vector<rsfde_stats> sb(h->count);
  for (int m = 0; m < M; ++m) {
    if (h->batched) {
      for (int i = 0; i < h->count; ++i) {
        Inst& I = h->inst[i];
        const double th = (m0 + m + 0.5) * I.p.dt;
        if (sample) {
          if (sample(ctx, i, th, I.e, I.f, (void*)h->stream) != 0) return RSFDE_E_INVALID_ARG;
        } else {
          CKS(builtin_sample(h, I, th, true));
        }
        ep[i] = I.e;
        fp[i] = I.f;
      }
      memset(sb.data(), 0, sizeof(rsfde_stats) * h->count);
      const int s = step_batched(h, ep.data(), fp.data(), u, sb.data());
      if (s < 0) return s;
      if (s > worst) worst = s;
      if (stats)
        for (int i = 0; i < h->count; ++i) {
          stats[i].iters += sb[i].iters;
          stats[i].cycles += sb[i].cycles;
          stats[i].outer_sweeps += sb[i].outer_sweeps;
          stats[i].converged = (m == 0 ? 1 : stats[i].converged) & sb[i].converged;
          stats[i].beta0 = sb[i].beta0;
          stats[i].rel_pres = sb[i].rel_pres;
          stats[i].rel_true_res = sb[i].rel_true_res;
        }
      continue;
    }
    for (int i = 0; i < h->count; ++i) {
      Inst& I = h->inst[i];
      const double th = (m0 + m + 0.5) * I.p.dt;
      if (sample) {
        if (sample(ctx, i, th, I.e, I.f, (void*)h->stream) != 0) return RSFDE_E_INVALID_ARG;
      } else {
        CKS(builtin_sample(h, I, th, true));
      }
      rsfde_stats s1;
      memset(&s1, 0, sizeof(s1));
      const int s = step_one(h, I, I.e, I.f, u[i], &s1);
      if (s < 0) return s;
      if (s > worst) worst = s;
      if (stats) {
        stats[i].iters += s1.iters;
        stats[i].cycles += s1.cycles;
        stats[i].outer_sweeps += s1.outer_sweeps;
        stats[i].converged = (m == 0 ? 1 : stats[i].converged) & s1.converged;
        stats[i].beta0 = s1.beta0;
        stats[i].rel_pres = s1.rel_pres;
        stats[i].rel_true_res = s1.rel_true_res;
      }
    }
  }
  CK(hipStreamSynchronize(h->stream));
  return worst;
}

int rsfde_destroy(rsfde_handle h) {
  if (!h) return RSFDE_E_INVALID_ARG;
  (void)hipStreamSynchronize(h->stream);
  for (auto& tp : h->pending) {
    (void)hipEventDestroy(tp.a);
    (void)hipEventDestroy(tp.b);
  }
  for (auto ev : h->ev_free) (void)hipEventDestroy(ev);
  if (h->sync_ev) (void)hipEventDestroy(h->sync_ev);
  for (auto& I : h->inst) graphs_clear(I.gexec);
  graphs_clear(h->bgexec);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->bhost) (void)hipHostFree(h->bhost);
  if (h->psum) (void)hipHostFree(h->psum);
  if (h->pmask) (void)hipHostFree(h->pmask);
  delete h;
  return RSFDE_OK;
}

const char* rsfde_strerror(int status) {
  switch (status) {
    case RSFDE_OK:
      return "ok";
    case RSFDE_W_NOT_CONVERGED:
      return "GMRES did not reach the tolerance within the allowed cycles (last iterate returned)";
    case RSFDE_E_INVALID_ARG:
      return "invalid argument";
    case RSFDE_E_WORKSPACE:
      return "workspace missing, misaligned (256 B) or too small";
    case RSFDE_E_HIP:
      snprintf(g_msg, sizeof(g_msg), "HIP runtime error: %s", hipGetErrorString(g_last_hip));
      return g_msg;
    case RSFDE_E_NONFINITE:
      return "non-finite residual norm";
    case RSFDE_E_UNSUPPORTED:
      return "grid size not supported: N_i + 1 must be 2^p or 3*2^p with 8 <= 2(N_i+1) <= 4096";
    case RSFDE_E_STATE:
      return "call order: ebar (e_min/e_max) or the fields are not set";
    default:
      return "unknown status";
  }
}

int rsfde_set_fields(rsfde_handle h, int instance, const rsfde_field* e, const rsfde_field* f,
                     const rsfde_field* psi) {
  if (h) h->fjob_key.clear();  // batched field jobs are rebuilt
  if (!h || instance < 0 || instance >= h->count || !e || !f || !psi) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  const int d = I.d;
  auto chk = [&](const rsfde_field* F, int lo, int hi) -> bool {
    if (F->kind < lo || F->kind > hi) return false;
    if (F->kind == RSFDE_FIELD_SINE_FIELD || F->kind == RSFDE_FIELD_SINE_MODES) {
      if (F->modes < 1 || F->modes > RSFDE_MAXMODES || !F->amp) return false;
    }
    return true;
  };
  if (!chk(e, RSFDE_FIELD_CONST, RSFDE_FIELD_SINE_FIELD)) return RSFDE_E_INVALID_ARG;
  if (!(f->kind == RSFDE_FIELD_ZERO || f->kind == RSFDE_FIELD_MANUFACTURED || f->kind == RSFDE_FIELD_SINE_MODES) ||
      !chk(f, 0, 7))
    return RSFDE_E_INVALID_ARG;
  if (!(psi->kind == RSFDE_FIELD_ZERO || psi->kind == RSFDE_FIELD_MANUFACTURED)) return RSFDE_E_INVALID_ARG;
  if (f->kind == RSFDE_FIELD_MANUFACTURED) {
    const double a = f->c[1];
    if (!(a >= 2.0 && a <= 6.0 && a == floor(a))) return RSFDE_E_INVALID_ARG;
    for (int i = 0; i < d; ++i)
      if (I.p.lo[i] != 0.0 || I.p.hi[i] != 1.0) return RSFDE_E_INVALID_ARG;
  }
  if (psi->kind == RSFDE_FIELD_MANUFACTURED) {
    const double a = psi->c[1];
    if (!(a >= 1.0 && a <= 6.0 && a == floor(a))) return RSFDE_E_INVALID_ARG;
  }
  if (e->kind == RSFDE_FIELD_SUMSQ_EXP && !(e->c[0] != 0.0)) return RSFDE_E_INVALID_ARG;
  auto load = [&](FieldHost& H, const rsfde_field* F) {
    H.spec = *F;
    H.amp.clear();
    if (F->amp && F->modes > 0) {
      int64_t cnt = 1;
      for (int i = 0; i < d; ++i) cnt *= F->modes;
      H.amp.assign(F->amp, F->amp + cnt);
    }
    H.spec.amp = nullptr;
    H.set = true;
    H.evaluated = false;
  };
  load(I.fe, e);
  load(I.ff, f);
  load(I.fpsi, psi);
  // device tables
  if (!I.fe.amp.empty())
    CK(hipMemcpyAsync(I.famp_e, I.fe.amp.data(), I.fe.amp.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  if (!I.ff.amp.empty())
    CK(hipMemcpyAsync(I.famp_f, I.ff.amp.data(), I.ff.amp.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  for (int i = 0; i < d; ++i) {
    if (I.fe.spec.modes > 0)
      CK(fields_sintab(I.fe.spec.modes, I.ax[i].N + 2, I.p.lo[i], I.ax[i].h, I.fsin_e[i], h->stream));
    if (I.ff.spec.modes > 0)
      CK(fields_sintab(I.ff.spec.modes, I.ax[i].N + 2, I.p.lo[i], I.ax[i].h, I.fsin_f[i], h->stream));
  }
  // manufactured source: coefficients of x^a (1-x)^a and its mirror, times the
  // Riemann-Liouville power-rule factors Gamma(k+1)/Gamma(k+1-alpha)
  std::vector<double> mc(3 * RSFDE_MC_STRIDE, 0.0);
  if (f->kind == RSFDE_FIELD_MANUFACTURED) {
    const int a = (int)llround(f->c[1]);
    std::vector<double> c(2 * a + 1, 0.0);
    double binom = 1.0;
    for (int j = 0; j <= a; ++j) {
      c[a + j] = (j % 2 ? -1.0 : 1.0) * binom;
      binom = binom * (a - j) / (j + 1);
    }
    for (int i = 0; i < d; ++i) {
      const double al = I.p.alpha[i];
      double* row = mc.data() + i * RSFDE_MC_STRIDE;
      for (int k = 0; k <= 2 * a; ++k) {
        if (c[k] == 0.0) continue;
        const double g = tgamma(k + 1.0) / tgamma(k + 1.0 - al);
        row[k] = c[k] * g;       // left-sided, power x^{k-alpha}
        row[13 + k] = c[k] * g;  // right-sided: p(1-y) = p(y) for this family
      }
      row[26] = -1.0 / (2.0 * cos(al * M_PI / 2.0));
      row[27] = al;
    }
  }
  CK(hipMemcpyAsync(I.fmc, mc.data(), mc.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  {
    // one-coordinate factors of the separable fields, once per closure point
    FieldDev fe = field_dev(I, I.fe, true), ff = field_dev(I, I.ff, false), fp = field_dev(I, I.fpsi, false);
    fp.a = (int)llround(I.fpsi.spec.c[1]);
    const GridDev gc = grid_dev(I, true);
    for (int i = 0; i < d; ++i) CK(fields_axis_tables(fe, ff, fp, gc, i, I.fax[i], h->stream));
  }
  CK(hipStreamSynchronize(h->stream));
  return RSFDE_OK;
}

int rsfde_eval_field(rsfde_handle h, int instance, int which, double t, double* out) {
  if (!h || instance < 0 || instance >= h->count || !out) return RSFDE_E_INVALID_ARG;
  if (which < RSFDE_WHICH_E || which > RSFDE_WHICH_PSI) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  if (!I.fe.set) return RSFDE_E_STATE;
  return eval_field(h, I, which, t, out);
}

int rsfde_eval_field_batch(rsfde_handle h, int which, double t, double* const* out) {
  if (!h || !out) return RSFDE_E_INVALID_ARG;
  if (which < RSFDE_WHICH_E || which > RSFDE_WHICH_PSI) return RSFDE_E_INVALID_ARG;
  for (int i = 0; i < h->count; ++i) {
    if (!out[i]) return RSFDE_E_INVALID_ARG;
    if (!h->inst[i].fe.set) return RSFDE_E_STATE;
  }
  if (h->count == 1 || !h->bdev) {
    for (int i = 0; i < h->count; ++i) CKS(eval_field(h, h->inst[i], which, t, out[i]));
    return RSFDE_OK;
  }
  std::vector<const void*> key(out, out + h->count);
  if (key != h->fjob_key || which != h->fjob_which) {
    CK(hipStreamSynchronize(h->stream));  // the staging area is free
    h->fjob_key.clear();
    h->rg[2].fill = 0;
    std::vector<FieldJob> jobs;
    std::vector<int> start(1, 0);
    for (int i = 0; i < h->count; ++i) {
      Inst& I = h->inst[i];
      FieldJob J;
      memset(&J, 0, sizeof(J));
      J.e = field_dev(I, I.fe, true);
      J.f = field_dev(I, which == RSFDE_WHICH_PSI ? I.fpsi : I.ff, false);
      if (which == RSFDE_WHICH_PSI) J.f.a = (int)llround(I.fpsi.spec.c[1]);
      J.g = grid_dev(I, which == RSFDE_WHICH_F);
      J.which = which;
      J.out = out[i];
      jobs.push_back(J);
      start.push_back(start.back() + (int)((J.g.size + 255) / 256));
    }
    h->fjob_dev = (const FieldJob*)bappend(h, 2, jobs.data(), jobs.size() * sizeof(FieldJob));
    h->fjob_start = (const int*)bappend(h, 2, start.data(), start.size() * sizeof(int));
    if (!h->fjob_dev || !h->fjob_start) return RSFDE_E_WORKSPACE;
    h->fjob_blocks = start.back();
    CK(bupload(h, 2));
    h->fjob_key = key;
    h->fjob_which = which;
  }
  CK(fields_eval_batched(h->fjob_dev, h->fjob_start, h->count, h->fjob_blocks, t, h->stream));
  return RSFDE_OK;
}

int rsfde_apply_A(rsfde_handle h, int instance, const double* e, const double* v, double* out) {
  if (!h || instance < 0 || instance >= h->count || !e || !v || !out) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  I.ecur = e;
  return run_chain(h, I, CH_APPLY_A, false, v, nullptr, nullptr, 0.0, out);
}

int rsfde_apply_prec(rsfde_handle h, int instance, const double* r, double* out) {
  if (!h || instance < 0 || instance >= h->count || !r || !out) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  if (!I.ebar_set) return RSFDE_E_STATE;
  return run_prec(h, I, false, r, out);
}

int rsfde_apply_prec_noalloc(rsfde_handle h, int instance, const double* r, double* out) {
  if (!h || instance < 0 || instance >= h->count || !r || !out) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  if (!I.ebar_set) return RSFDE_E_STATE;
  // temporaries: 2 (d - 1) FP64 vectors, each starting on a 256-byte boundary
  const int ntemp = I.d == 1 ? 0 : (I.d == 2 ? 2 : 4);
  const size_t vec = ((size_t)I.n * sizeof(double) + 255) & ~(size_t)255;
  if ((size_t)ntemp * vec > (size_t)RSFDE_NOALLOC_SCRATCH_BYTES) return RSFDE_E_WORKSPACE;
  void* base = nullptr;
  CK(scratch_ptr(&base));
  void* T[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < ntemp; ++k) T[k] = (char*)base + (size_t)k * vec;
  // no event creation either: kernel timing is suspended for this call
  const unsigned mask = h->tmask;
  h->tmask = 0;
  const int st = run_prec(h, I, false, r, out, PM_BP_INV, nullptr, T);
  h->tmask = mask;
  return st;
}

int rsfde_apply_prec_form(rsfde_handle h, int instance, int form, const double* r, double* out) {
  if (!h || instance < 0 || instance >= h->count || !r || !out) return RSFDE_E_INVALID_ARG;
  if (form != RSFDE_PREC_BP_INV && form != RSFDE_PREC_PHALF_BINV && form != RSFDE_PREC_PHALF &&
      form != RSFDE_PREC_STRANG)
    return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  if (!I.ebar_set) return RSFDE_E_STATE;
  if (form == RSFDE_PREC_STRANG) {
    if (I.p.method != RSFDE_SPGM) return RSFDE_E_STATE;  // its tables exist in that form only
    return run_strang_prec(h, I, r, -1, out);
  }
  const int pm = form == RSFDE_PREC_BP_INV ? PM_BP_INV : (form == RSFDE_PREC_PHALF_BINV ? PM_PH_BINV : PM_PH);
  return run_prec(h, I, false, r, out, pm);
}

int rsfde_compute_F(rsfde_handle h, int instance, const double* f_closure, double* out) {
  if (!h || instance < 0 || instance >= h->count || !f_closure || !out) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  double al[3] = {I.p.alpha[0], I.p.alpha[1], I.p.alpha[2]};
  CK(compute_F(f_closure, grid_dev(I, false), al, out, h->stream));
  return RSFDE_OK;
}

int rsfde_rhs(rsfde_handle h, int instance, const double* e, const double* F, const double* u,
              double* out) {
  if (!h || instance < 0 || instance >= h->count || !e || !F || !u || !out) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  I.ecur = e;
  return run_chain(h, I, CH_RHS, false, u, nullptr, F, I.p.dt, out);
}

int rsfde_get_tables(rsfde_handle h, int instance, int axis, double* s, double* q, double* lambda) {
  if (!h || instance < 0 || instance >= h->count) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  if (axis < 0 || axis >= I.d) return RSFDE_E_INVALID_ARG;
  const Axis& A = I.ax[axis];
  CK(hipStreamSynchronize(h->stream));
  if (s) CK(hipMemcpy(s, A.s, A.N * sizeof(double), hipMemcpyDeviceToHost));
  if (q) CK(hipMemcpy(q, A.q, A.N * sizeof(double), hipMemcpyDeviceToHost));
  if (lambda) CK(hipMemcpy(lambda, A.lam64, A.N * sizeof(double), hipMemcpyDeviceToHost));
  return RSFDE_OK;
}

int rsfde_get_pass_shape(rsfde_handle h, int instance, int axis, int precision, int transform,
                         int* length, int* per_workgroup) {
  if (!h || instance < 0 || instance >= h->count || !length || !per_workgroup) return RSFDE_E_INVALID_ARG;
  const Inst& I = h->inst[instance];
  if (axis < 0 || axis >= I.d || (transform != 0 && transform != 1)) return RSFDE_E_INVALID_ARG;
  if (precision != RSFDE_FP64 && precision != RSFDE_MIXED) return RSFDE_E_INVALID_ARG;
  const bool fp32 = precision == RSFDE_MIXED;
  if (fp32 && I.p.precision != RSFDE_MIXED) return RSFDE_E_INVALID_ARG;
  const int L = I.ax[axis].L;
  int nt = 0, ppt = 0;
  pass_shape_rt(L, fp32, axis > 0, I.var[axis][fp32 ? 1 : 0][transform], &nt, &ppt);
  *length = L;
  *per_workgroup = ppt / 2;
  return RSFDE_OK;
}

int rsfde_get_pass_plan(rsfde_handle h, int instance, int axis, int precision, int transform,
                        int* code, int* radices, int* nstage) {
  if (!h || instance < 0 || instance >= h->count || !code || !radices || !nstage)
    return RSFDE_E_INVALID_ARG;
  const Inst& I = h->inst[instance];
  if (axis < 0 || axis >= I.d || (transform != 0 && transform != 1)) return RSFDE_E_INVALID_ARG;
  if (precision != RSFDE_FP64 && precision != RSFDE_MIXED) return RSFDE_E_INVALID_ARG;
  const bool fp32 = precision == RSFDE_MIXED;
  if (fp32 && I.p.precision != RSFDE_MIXED) return RSFDE_E_INVALID_ARG;
  if (!pass_plan_rt(I.ax[axis].L, I.var[axis][fp32 ? 1 : 0][transform], code, radices, nstage))
    return RSFDE_E_INVALID_ARG;
  return RSFDE_OK;
}

int rsfde_set_graph(rsfde_handle h, int enable) {
  if (!h || (enable != 0 && enable != 1)) return RSFDE_E_INVALID_ARG;
  if (enable && !h->cap) CK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  if (!enable) {
    CK(hipStreamSynchronize(h->stream));
    for (auto& I : h->inst) graphs_clear(I.gexec);
    graphs_clear(h->bgexec);
  }
  h->graphs = enable != 0;
  return RSFDE_OK;
}

int rsfde_set_true_residual(rsfde_handle h, int enable) {
  if (!h || (enable != 0 && enable != 1)) return RSFDE_E_INVALID_ARG;
  h->true_res = enable != 0;
  return RSFDE_OK;
}

int rsfde_set_timing(rsfde_handle h, unsigned mask, int every) {
  if (!h || every < 1) return RSFDE_E_INVALID_ARG;
  CK(hipStreamSynchronize(h->stream));
  CKS(flush_timing(h));
  h->tmask = mask;
  h->tevery = every;
  for (int c = 0; c < RSFDE_K_NCLASS; ++c) {
    h->tseen[c] = 0;
    h->t_launches[c] = 0;
    h->t_ms[c] = 0;
    h->t_bytes[c] = 0;
  }
  return RSFDE_OK;
}

int rsfde_get_timing(rsfde_handle h, int kclass, long long* launches, double* ms, double* bytes) {
  if (!h || kclass < 0 || kclass >= RSFDE_K_NCLASS) return RSFDE_E_INVALID_ARG;
  CK(hipStreamSynchronize(h->stream));
  CKS(flush_timing(h));
  if (launches) *launches = h->t_launches[kclass];
  if (ms) *ms = h->t_ms[kclass];
  if (bytes) *bytes = h->t_bytes[kclass];
  return RSFDE_OK;
}

int rsfde_prescan_ebar(rsfde_handle h, int instance, int M) {
  if (!h || instance < 0 || instance >= h->count || M < 1) return RSFDE_E_INVALID_ARG;
  Inst& I = h->inst[instance];
  if (!I.fe.set) return RSFDE_E_STATE;
  CK(minmax_reset(I.eminmax, h->stream));
  const int scans = I.fe.spec.time_dependent ? M : 1;
  for (int m = 0; m < scans; ++m) {
    CKS(eval_field(h, I, RSFDE_WHICH_E, (m + 0.5) * I.p.dt, I.e));
    CK(minmax_accum(I.e, I.n, I.eminmax, I.partial, I.counters + 2, h->stream));
  }
  I.fe.evaluated = false;
  double mm[2];
  CK(hipMemcpyAsync(mm, I.eminmax, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  CK(hipStreamSynchronize(h->stream));
  if (!(mm[0] > 0.0) || !isfinite(mm[1])) return RSFDE_E_INVALID_ARG;
  return rsfde_set_ebar(h, instance, mm[0], mm[1]);
}

}  // extern "C"
