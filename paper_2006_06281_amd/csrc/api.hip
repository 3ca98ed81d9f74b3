// Host runtime behind the C ABI of fastcpd.h: argument validation, the
// workspace carve-up, the per-handle state machine and the order of kernel
// launches inside one EM iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fastcpd.h"
#include "common.hpp"
#include "eig.hpp"
#include "kernels.hpp"
#include "net.hpp"
#include "orig.hpp"
#include "lowrank.hpp"

using namespace fcpd;

namespace {

thread_local std::string g_last_error;

// Size of the static device scratch behind cpdnet_forward_noalloc.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

enum class Stage { Init = 0, Prepared = 1 };

struct Region {
  size_t off = 0, bytes = 0;
};

// Byte offsets of every buffer inside the caller's workspace.
struct Layout {
  size_t total = 0;
  Region sc, X, Xt, Xnew, Y, W, xs, ys, Yt, P1, tbar, partA, partB, nnY, nnX, llpart,
      sigpart, initpart, featX, featY, featV;
  Region permX, permY, invY, keys, bbox, boxX, boxY, logdtmp, Xraw;  // spatial order / culling
  bool sorted = false, cull = false;
  bool eig_shared = false;  // batch member: U64 and eigen-prep scratch live in a shared slot
  Region U, lam, U64, tpart, GT, HT;
  EigLayout eig;
  OrigLayout orig;
  LowRankLayout lr;
  int splitsA = 1, chunkA = 1, splitsB = 1, chunkB = 1;
  int mchunks = 1, mrows = 64;
  int Kcap = 0;
};

size_t add(Layout& L, Region& r, size_t bytes) {
  r.off = L.total;
  r.bytes = bytes;
  L.total += (bytes + 255) & ~(size_t)255;
  return r.off;
}

int kcap_of(const cpd_params& p) {
  if (p.method == CPD_METHOD_ORIGINAL) return 0;
  if (p.eig_mode == CPD_EIG_FULL) return eig_full_capacity(p.M);
  return p.K;
}

// A batch member sizes its E-step partials for a fixed split length
// (batch_chunk points per split) instead of the single-instance plan.
void chunk_plan(int M, int N, int chunk, int* splitsA, int* chunkA, int* splitsB, int* chunkB) {
  *chunkA = std::min(chunk, (M + 3) & ~3);
  *splitsA = (M + *chunkA - 1) / *chunkA;
  *chunkB = std::min(chunk, (N + 3) & ~3);
  *splitsB = (N + *chunkB - 1) / *chunkB;
}

template <typename T>
Layout make_layout(const cpd_params& p, int batch_chunk = 0) {
  Layout L;
  const size_t M = (size_t)p.M, N = (size_t)p.N;
  const size_t p4 = sizeof(P4<T>);
  if (batch_chunk > 0)
    chunk_plan(p.M, p.N, batch_chunk, &L.splitsA, &L.chunkA, &L.splitsB, &L.chunkB);
  else if (p.precision == CPD_PREC_BF16X)
    bfx_splits(p.M, p.N, 0, &L.splitsA, &L.chunkA, &L.splitsB, &L.chunkB);
  else
    estep_splits<T>(p.M, p.N, &L.splitsA, &L.chunkA, &L.splitsB, &L.chunkB);
  const size_t M256 = (size_t)pad256(p.M), N256 = (size_t)pad256(p.N);
  add(L, L.sc, sizeof(DevScalars));
  add(L, L.X, M * p4);
  add(L, L.Xt, M * p4);
  add(L, L.Xnew, M * p4);
  add(L, L.Y, N * p4);
  add(L, L.W, M * p4);
  add(L, L.xs, M256 * p4);
  add(L, L.ys, N256 * p4);
  if (p.precision == CPD_PREC_BF16X) {
    add(L, L.featX, M256 * 64);
    add(L, L.featY, N256 * 64);
    add(L, L.featV, N256 * 64);
  }
  add(L, L.Yt, M * p4);
  add(L, L.P1, M * sizeof(T));
  add(L, L.tbar, M * sizeof(T));
  add(L, L.partA, (size_t)L.splitsA * N * sizeof(T));
  // (BF16X: room for the most splits cpd_init may fit to the device)
  const int splitsB_cap = (batch_chunk == 0 && p.precision == CPD_PREC_BF16X)
                              ? std::max(L.splitsB, bfx_splitsB_max(p.M, p.N))
                              : L.splitsB;
  add(L, L.partB, (size_t)splitsB_cap * 5 * M * sizeof(T));
  // nearest-neighbour indices of the two-way matching (per scene / model point)
  add(L, L.nnY, N * sizeof(int));
  add(L, L.nnX, M * sizeof(int));
  add(L, L.llpart, ((N + 255) / 256) * sizeof(double));
  // sigma^2 partials: per 256 rows (k_sig_part) or per 64 (fused into the M-step)
  add(L, L.sigpart, 2 * (size_t)std::max(sigma2_blocks<T>(p.M), (p.M + 63) / 64) * sizeof(double));
  add(L, L.initpart, 8 * (size_t)init_blocks(p.M, p.N) * sizeof(double));
  // Points are kept in Hilbert order (single handles and batch members alike).
  L.sorted = !(p.flags & CPD_FLAG_NO_SORT);
  L.cull = L.sorted && !(p.flags & CPD_FLAG_NO_CULL);
  if (L.sorted) {
    size_t n2 = 1;
    while (n2 < std::max(M, N)) n2 <<= 1;
    add(L, L.permX, M * sizeof(int));
    add(L, L.permY, N * sizeof(int));
    add(L, L.invY, N * sizeof(int));
    add(L, L.keys, n2 * sizeof(unsigned long long));
    add(L, L.bbox, (size_t)order_bbox_doubles(p.M + p.N) * sizeof(double));
    add(L, L.logdtmp, N * sizeof(T));
    add(L, L.Xraw, M * p4);
  }
  if (L.cull) {
    // boxes of 64-point tiles (FP32 / FP64 E-step) or 16-point tiles (BF16X)
    add(L, L.boxX, 2 * ((M + 15) / 16) * p4);
    add(L, L.boxY, 2 * ((N + 15) / 16) * p4);
  }
  L.Kcap = kcap_of(p);
  if (p.method != CPD_METHOD_ORIGINAL) {  // FAST and CPD-L keep eigenpairs
    const size_t K = (size_t)L.Kcap;
    L.mchunks = fast_mstep_chunks<T>(p.M, &L.mrows);
    add(L, L.U, M * K * sizeof(T));
    add(L, L.lam, K * sizeof(double));
    // A batch member needs its FP64 eigenvectors and the solver's scratch
    // only while it prepares: they come from one of the batch's per-thread
    // slots (eig_slot_bytes) instead of the member's own workspace.
    L.eig_shared = batch_chunk > 0 && p.eig_mode != CPD_EIG_IMPORT;
    if (!L.eig_shared) add(L, L.U64, M * K * sizeof(double));
    add(L, L.tpart, (size_t)L.mchunks * K * 4 * sizeof(T));
    add(L, L.GT, K * p4);
    add(L, L.HT, K * p4);
    if (p.eig_mode != CPD_EIG_IMPORT && !L.eig_shared) {
      L.eig = eig_layout(p.M, p.eig_mode, p.K, p.oversample, L.total);
      L.total = L.eig.end;
    }
    // the K x K system: CPD-L's M-step, and the matched solve of two-way
    // registration on a single Fast handle
    if (p.method == CPD_METHOD_ORIGINAL_LOWRANK || batch_chunk == 0) {
      L.lr = lowrank_layout(p.M, L.Kcap, L.total);
      L.total = L.lr.end;
    }
  } else {
    L.orig = orig_layout(p.M, (int)sizeof(T), L.total);
    L.total = L.orig.end;
  }
  return L;
}

// Bytes of a shared eigen-prep slot for one batch member: its FP64
// eigenvectors (M x Kcap) followed by the solver's scratch.
size_t eig_slot_u64_bytes(const cpd_params& p) {
  return ((size_t)p.M * kcap_of(p) * sizeof(double) + 255) & ~(size_t)255;
}
size_t eig_slot_bytes(const cpd_params& p) {
  return eig_layout(p.M, p.eig_mode, p.K, p.oversample, eig_slot_u64_bytes(p)).end;
}

Layout layout_for(const cpd_params& p, int batch_chunk = 0) {
  return p.precision == CPD_PREC_FP64 ? make_layout<double>(p, batch_chunk)
                                      : make_layout<float>(p, batch_chunk);
}

}  // namespace

struct cpd_ctx {
  cpd_params p{};
  Layout L;
  char* ws = nullptr;
  hipStream_t st = nullptr;
  Stage stage = Stage::Init;
  int K = 0;  // eigenpairs held
  int sig_fused = 0;  // sigma^2 partials the last enqueued M-step wrote (0: none)
  double t_eig = 0.0;
  std::string err;
  JacobiBatcher* jb = nullptr;  // set while a batch prepares: grouped Jacobi solves
  char* eig_slot = nullptr;     // set while a batch prepares: shared U64 + solver scratch
  DevScalars* host_sc = nullptr;  // pinned host copies of the scalars (two slots), lazily made
  ~cpd_ctx() {
    if (host_sc) (void)hipHostFree(host_sc);
  }
  template <typename U> U* at(const Region& r) const { return reinterpret_cast<U*>(ws + r.off); }
  DevScalars* sc() const { return at<DevScalars>(L.sc); }
  // caller row of internal model / scene row i (NULL: same order)
  const int* permX() const { return L.sorted ? at<int>(L.permX) : nullptr; }
  const int* permY() const { return L.sorted ? at<int>(L.permY) : nullptr; }
  const int* invY() const { return L.sorted ? at<int>(L.invY) : nullptr; }
  // device address of the iteration frame's origin (NULL: the caller's frame)
  const double* origin() const { return L.sorted ? sc()->origin : nullptr; }
  // model points in the caller's frame (internal order), for the Gram matrix
  template <typename T> const P4<T>* Xgram() const { return at<P4<T>>(L.sorted ? L.Xraw : L.X); }
};

namespace {

// Events that only time work on the handle's stream: recorded without the
// system-scope fence (an L2 write-back and invalidation), which would make the
// kernel after each event start from a cold cache and slow the timed run.
constexpr unsigned kTimingEventFlags = hipEventDisableSystemFence;

// A HIP event released when the guard leaves scope.
struct EventGuard {
  hipEvent_t e = nullptr;
  ~EventGuard() {
    if (e) (void)hipEventDestroy(e);
  }
};

cpd_status fail(cpd_ctx* h, cpd_status s, const std::string& msg) {
  g_last_error = msg;
  if (h) h->err = msg;
  return s;
}

cpd_status hip_fail(cpd_ctx* h, hipError_t e, const char* what) {
  return fail(h, CPD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                       \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call);    \
  } while (0)

cpd_status validate(const cpd_params* p) {
  if (!p) return fail(nullptr, CPD_E_ARG, "params is NULL");
  if (p->abi_version != CPD_ABI_VERSION) return fail(nullptr, CPD_E_ARG, "abi_version mismatch");
  if (p->M < 1 || p->N < 1 || p->M > (1 << 26) || p->N > (1 << 26))
    return fail(nullptr, CPD_E_ARG, "M and N must be in [1, 2^26]");
  if (p->D < 1 || p->D > 3) return fail(nullptr, CPD_E_ARG, "D must be 1, 2 or 3");
  if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(nullptr, CPD_E_ARG, "beta must be > 0");
  if (!(p->lambda > 0.0) || !std::isfinite(p->lambda))
    return fail(nullptr, CPD_E_ARG, "lambda must be > 0");
  if (!(p->w >= 0.0 && p->w < 1.0)) return fail(nullptr, CPD_E_ARG, "w must satisfy 0 <= w < 1");
  if (!std::isfinite(p->sigma2_init)) return fail(nullptr, CPD_E_ARG, "sigma2_init not finite");
  if (p->method != CPD_METHOD_ORIGINAL && p->method != CPD_METHOD_FAST &&
      p->method != CPD_METHOD_ORIGINAL_LOWRANK)
    return fail(nullptr, CPD_E_ARG, "unknown method");
  if (p->precision < CPD_PREC_FP64 || p->precision > CPD_PREC_BF16X)
    return fail(nullptr, CPD_E_ARG, "unknown precision");
  if (p->method != CPD_METHOD_ORIGINAL) {
    if (p->eig_mode < CPD_EIG_FULL || p->eig_mode > CPD_EIG_IMPORT)
      return fail(nullptr, CPD_E_ARG, "unknown eig_mode");
    if (p->eig_mode != CPD_EIG_FULL && (p->K < 1 || p->K > p->M))
      return fail(nullptr, CPD_E_ARG, "K must be in [1, M]");
    if (p->eig_mode == CPD_EIG_TOPK) {
      const int over = p->oversample > 0 ? p->oversample : 20;
      if (p->K + over > p->M) return fail(nullptr, CPD_E_ARG, "K + oversample must not exceed M");
      if (p->K + over > eig_topk_max_cols())
        return fail(nullptr, CPD_E_UNSUPPORTED, "K + oversample exceeds the randomized solver's width");
      if (p->power_iters > 16) return fail(nullptr, CPD_E_ARG, "power_iters must be <= 16");
    }
  }
  if (!(p->tol >= 0.0)) return fail(nullptr, CPD_E_ARG, "tol must be >= 0");
  if (p->max_iter < 1) return fail(nullptr, CPD_E_ARG, "max_iter must be >= 1");
  if (p->flags & ~(CPD_FLAG_NO_SORT | CPD_FLAG_NO_CULL))
    return fail(nullptr, CPD_E_ARG, "unknown bits in flags");
  if (p->precision == CPD_PREC_BF16X && p->method != CPD_METHOD_FAST)
    return fail(nullptr, CPD_E_UNSUPPORTED, "BF16X precision is implemented for the Fast method");
  if (p->precision == CPD_PREC_BF16X && p->D != 3)
    return fail(nullptr, CPD_E_UNSUPPORTED, "BF16X is implemented for D = 3");
  return CPD_OK;
}

cpd_status check_device(cpd_ctx* h) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) return fail(h, CPD_E_DEVICE, "no HIP device available");
  int dev = 0;
  HIPCHK(h, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(h, hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(h, CPD_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", need gfx950");
  return CPD_OK;
}

// ------------------------------------------------------------- one step
template <typename T>
void enqueue_estep(cpd_ctx* h, int gate, T* logd_out, hipEvent_t* ev = nullptr) {
  const Layout& L = h->L;
  EStepArgs<T> a{};
  a.Xt = h->at<P4<T>>(L.Xt);
  a.Y = h->at<P4<T>>(L.Y);
  a.xs = h->at<P4<T>>(L.xs);
  a.ys = h->at<P4<T>>(L.ys);
  a.M = h->p.M;
  a.N = h->p.N;
  a.D = h->p.D;
  a.w = h->p.w;
  a.sc = h->sc();
  a.gate = gate;
  a.splitsA = L.splitsA;
  a.chunkA = L.chunkA;
  a.splitsB = L.splitsB;
  a.chunkB = L.chunkB;
  a.partA = h->at<T>(L.partA);
  a.partB = h->at<T>(L.partB);
  a.llpart = h->at<double>(L.llpart);
  a.logd_out = logd_out;
  a.Yt = h->at<P4<T>>(L.Yt);
  a.P1 = h->at<T>(L.P1);
  a.tbar = h->at<T>(L.tbar);
  a.ev = ev;
  a.featX = h->at<__bf16>(L.featX);
  a.featY = h->at<__bf16>(L.featY);
  a.featV = h->at<__bf16>(L.featV);
  a.boxX = L.cull ? h->at<P4<T>>(L.boxX) : nullptr;
  a.boxY = L.cull ? h->at<P4<T>>(L.boxY) : nullptr;
  a.box_shift = h->p.precision == CPD_PREC_BF16X ? 4 : 6;
  a.featY_L = h->p.precision == CPD_PREC_BF16X ? a.featY : nullptr;
  if (h->p.precision == CPD_PREC_BF16X)
    estep_bf16x_launch(reinterpret_cast<const EStepArgs<float>&>(a), h->st);
  else
    estep_launch<T>(a, h->st);
}

template <typename T>
void enqueue_mstep(cpd_ctx* h, int gate) {
  const Layout& L = h->L;
  if (h->p.method == CPD_METHOD_FAST) {
    FastMArgs<T> a{};
    a.X = h->at<P4<T>>(L.X);
    a.Yt = h->at<P4<T>>(L.Yt);
    a.U = h->at<T>(L.U);
    a.lam = h->at<double>(L.lam);
    a.M = h->p.M;
    a.K = h->K;
    a.D = h->p.D;
    a.lmbda = h->p.lambda;
    a.sc = h->sc();
    a.gate = gate;
    a.rows_per_chunk = L.mrows;
    a.chunks = L.mchunks;
    a.tpart = h->at<T>(L.tpart);
    a.GT = h->at<P4<T>>(L.GT);
    a.HT = h->at<P4<T>>(L.HT);
    a.Xnew = h->at<P4<T>>(L.Xnew);
    a.W = h->at<P4<T>>(L.W);
    a.Xt = h->at<P4<T>>(L.Xt);
    a.tbar = h->at<T>(L.tbar);
    a.sigpart = h->at<double>(L.sigpart);
    h->sig_fused = fast_mstep_launch<T>(a, h->st);
  } else if (h->p.method == CPD_METHOD_ORIGINAL_LOWRANK) {
    LowRankArgs<T> a{};
    a.X = h->at<P4<T>>(L.X);
    a.Yt = h->at<P4<T>>(L.Yt);
    a.P1 = h->at<T>(L.P1);
    a.U64 = h->at<double>(L.U64);
    a.lam = h->at<double>(L.lam);
    a.M = h->p.M;
    a.K = h->K;
    a.lmbda = h->p.lambda;
    a.sc = h->sc();
    a.gate = gate;
    a.ws = h->ws;
    a.L = &L.lr;
    a.Xnew = h->at<P4<T>>(L.Xnew);
    a.W = h->at<P4<T>>(L.W);
    h->sig_fused = 0;
    lowrank_mstep_launch<T>(a, h->st);
  } else {
    OrigArgs<T> a{};
    a.X = h->at<P4<T>>(L.X);
    a.Yt = h->at<P4<T>>(L.Yt);
    a.P1 = h->at<T>(L.P1);
    a.M = h->p.M;
    a.D = h->p.D;
    a.lmbda = h->p.lambda;
    a.sc = h->sc();
    a.gate = gate;
    a.ws = h->ws;
    a.L = &L.orig;
    a.Xnew = h->at<P4<T>>(L.Xnew);
    a.W = h->at<P4<T>>(L.W);
    h->sig_fused = 0;
    orig_mstep_launch<T>(a, h->st);
  }
}

template <typename T>
void enqueue_sigma2(cpd_ctx* h, int gate) {
  const Layout& L = h->L;
  Sigma2Args<T> a{};
  a.Xt = h->at<P4<T>>(L.Xt);
  a.Xnew = h->at<P4<T>>(L.Xnew);
  a.Yt = h->at<P4<T>>(L.Yt);
  a.tbar = h->at<T>(L.tbar);
  a.P1 = h->p.method != CPD_METHOD_FAST ? h->at<T>(L.P1) : nullptr;  // N_P form
  a.M = h->p.M;
  a.N = h->p.N;
  a.D = h->p.D;
  a.w = h->p.w;
  a.sc = h->sc();
  a.gate = gate;
  a.part = h->at<double>(L.sigpart);
  a.blocks = sigma2_blocks<T>(h->p.M);
  if (h->sig_fused > 0) {  // the M-step already wrote the partials
    a.fused = 1;
    a.blocks = h->sig_fused;
  }
  a.llpart = h->at<double>(L.llpart);
  a.llblocks = (h->p.N + 255) / 256;
  sigma2_launch<T>(a, h->st);
}

// E-step start, M-step start, M-step end (the paper's t_c and t_iter).
struct PhaseEvents {
  hipEvent_t e[3];
};

template <typename T>
void enqueue_step(cpd_ctx* h, int gate, PhaseEvents* ev) {
  if (ev) (void)hipEventRecord(ev->e[0], h->st);
  enqueue_estep<T>(h, gate, nullptr);
  if (ev) (void)hipEventRecord(ev->e[1], h->st);
  enqueue_mstep<T>(h, gate);
  if (ev) (void)hipEventRecord(ev->e[2], h->st);
  enqueue_sigma2<T>(h, gate);
}

__global__ void k_arm(DevScalars* sc, int reset_iter) {
  if (threadIdx.x == 0) {
    sc->done = 0;
    sc->converged = 0;
    if (reset_iter) sc->iter = 0;
  }
}

cpd_status ready_for_steps(cpd_ctx* h) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  if (h->stage != Stage::Prepared)
    return fail(h, CPD_E_STATE, "cpd_eig_prepare must run before stepping");
  return CPD_OK;
}

template <typename T>
cpd_status step_impl(cpd_ctx* h, cpd_step_info* info) {
  // ungated: every kernel of the step runs whatever sc->done holds (only
  // cpd_register reads that flag, and it re-arms it), so nothing is reset
  enqueue_step<T>(h, 0, nullptr);
  HIPCHK(h, hipGetLastError());
  if (!info) return CPD_OK;
  DevScalars s;
  HIPCHK(h, hipMemcpyAsync(&s, h->sc(), sizeof(s), hipMemcpyDeviceToHost, h->st));
  HIPCHK(h, hipStreamSynchronize(h->st));
  info->iter = s.iter;
  info->converged = s.converged;
  info->sigma2 = s.sigma2;
  info->dsigma2 = s.dsigma2;
  info->loglik = s.loglik;
  if (s.nonfinite == 2) return fail(h, CPD_E_NUMERIC, "Cholesky factorisation broke down");
  if (s.nonfinite) return fail(h, CPD_E_NUMERIC, "sigma^2 became non-finite");
  return CPD_OK;
}

template <typename T>
cpd_status register_impl(cpd_ctx* h, const void* W0, void* X_out, void* W_out, cpd_result* res) {
  const Layout& L = h->L;
  const auto t0 = std::chrono::steady_clock::now();
  if (W0) {
    const T* w0 = static_cast<const T*>(W0);
    if (h->permX()) {  // into internal order (Xnew is free before the first step)
      T* tmp = h->at<T>(L.Xnew);
      gather_rows_launch<T>(w0, tmp, h->permX(), h->p.M, h->p.D, h->st);
      w0 = tmp;
    }
    phi_apply_launch<T>(h->at<P4<T>>(L.X), w0, h->at<P4<T>>(L.Xt), h->p.M,
                        h->p.D, h->p.beta, h->st);
    // sigma^2 of the warm start: the closed form at X + Phi W0, or the
    // caller's sigma2_init (never the previous run's value)
    reset_sigma2_launch<T>(h->at<P4<T>>(L.Xt), h->at<P4<T>>(L.Y), h->p.M, h->p.N, h->p.D,
                           h->sc(), h->at<double>(L.initpart), h->st,
                           h->p.sigma2_init > 0.0 ? kS2Start : kS2Warm);
  }
  hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, h->st, h->sc(), 1);
  HIPCHK(h, hipGetLastError());
  if (!h->host_sc) {
    void* p = nullptr;
    HIPCHK(h, hipHostMalloc(&p, 2 * sizeof(DevScalars), hipHostMallocDefault));
    h->host_sc = static_cast<DevScalars*>(p);
  }
  // Iterations are enqueued in batches, each followed by a copy of the
  // scalars into its pinned slot.  Two batches are in flight: the host
  // enqueues the next batch before it waits for the previous one's copy, so
  // the device does not idle through the host's round trip.  After
  // convergence the launches still queued see sc->done and return at once.
  const int batch = 8;
  std::vector<EventGuard> guards(res ? 2 * 3 * batch : 0);
  std::vector<PhaseEvents> evs(res ? 2 * batch : 0);
  for (int i = 0; i < (int)guards.size(); ++i) {
    HIPCHK(h, hipEventCreateWithFlags(&guards[i].e, kTimingEventFlags));
    evs[i / 3].e[i % 3] = guards[i].e;
  }
  EventGuard copied[2];
  for (auto& g : copied) HIPCHK(h, hipEventCreateWithFlags(&g.e, hipEventDisableTiming));
  double t_c = 0, t_it = 0;
  DevScalars s{};
  cpd_status status = CPD_OK;
  int nbs[2] = {0, 0};
  int head = 0, inflight = 0, enqueued = 0;
  for (;;) {
    while (inflight < 2 && enqueued < h->p.max_iter) {
      const int slot = (head + inflight) & 1;
      const int nb = std::min(batch, h->p.max_iter - enqueued);
      for (int i = 0; i < nb; ++i)
        enqueue_step<T>(h, 1, res ? &evs[slot * batch + i] : nullptr);
      HIPCHK(h, hipGetLastError());
      HIPCHK(h, hipMemcpyAsync(&h->host_sc[slot], h->sc(), sizeof(DevScalars),
                               hipMemcpyDeviceToHost, h->st));
      HIPCHK(h, hipEventRecord(copied[slot].e, h->st));
      nbs[slot] = nb;
      enqueued += nb;
      ++inflight;
    }
    if (inflight == 0) break;
    HIPCHK(h, hipEventSynchronize(copied[head].e));
    s = h->host_sc[head];
    if (res) {
      for (int i = 0; i < nbs[head]; ++i) {
        const PhaseEvents& e = evs[head * batch + i];
        float a = 0, b = 0;
        (void)hipEventElapsedTime(&a, e.e[0], e.e[1]);
        (void)hipEventElapsedTime(&b, e.e[1], e.e[2]);
        t_c += a * 1e-3;
        t_it += b * 1e-3;
      }
    }
    head ^= 1;
    --inflight;
    if (s.done) break;
  }
  if (s.nonfinite == 2) status = fail(h, CPD_E_NUMERIC, "Cholesky factorisation broke down");
  else if (s.nonfinite) status = fail(h, CPD_E_NUMERIC, "sigma^2 became non-finite");
  if (X_out)
    unpack_launch<T>(h->at<P4<T>>(L.Xt), static_cast<T*>(X_out), h->p.M, h->p.D, h->st, h->permX(),
                     h->origin());
  if (W_out)
    unpack_launch<T>(h->at<P4<T>>(L.W), static_cast<T*>(W_out), h->p.M, h->p.D, h->st, h->permX());
  HIPCHK(h, hipStreamSynchronize(h->st));
  const double total =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (res) {
    res->iters = s.iter;
    res->converged = s.converged;
    res->sigma2 = s.sigma2;
    res->t_c = t_c;
    res->t_iter = t_it;
    res->t_eig = h->t_eig;
    res->t_o = std::max(0.0, total - t_c - t_it);
  }
  if (status != CPD_OK) return status;
  return s.converged ? CPD_OK : CPD_NOT_CONVERGED;
}

template <typename T>
cpd_status init_impl(cpd_ctx* h, const void* X, const void* Y) {
  const Layout& L = h->L;
  init_launch<T>(static_cast<const T*>(X), static_cast<const T*>(Y), h->at<P4<T>>(L.X),
                 h->at<P4<T>>(L.Xt), h->at<P4<T>>(L.Y), h->p.M, h->p.N, h->p.D, h->p.sigma2_init,
                 h->p.tol, h->p.max_iter, h->sc(), h->at<double>(L.initpart), h->st,
                 h->p.precision == CPD_PREC_BF16X ? kBfxSigma2FloorRel : 0.0);
  if (L.sorted) {
    // Hilbert order of X and Y (xs serves as the staging buffer: it holds
    // max(M, N) rounded up to 256 points and is cleared below); Xt = X.
    P4<T>* stage = h->at<P4<T>>(L.xs.bytes >= L.ys.bytes ? L.xs : L.ys);
    spatial_order_launch<T>(h->at<P4<T>>(L.X), h->p.M, h->at<P4<T>>(L.Y), h->p.N,
                            h->at<int>(L.permX), h->at<int>(L.permY), h->at<int>(L.invY),
                            h->at<unsigned long long>(L.keys), h->at<double>(L.bbox), stage,
                            h->at<P4<T>>(L.Xraw), h->sc(), h->st);
    HIPCHK(h, hipMemcpyAsync(h->ws + L.Xt.off, h->ws + L.X.off, L.X.bytes, hipMemcpyDeviceToDevice,
                             h->st));
  }
  // W starts at 0 (so Xt = X); the padding of the prescaled copies stays 0
  HIPCHK(h, hipMemsetAsync(h->ws + L.W.off, 0, L.W.bytes, h->st));
  HIPCHK(h, hipMemsetAsync(h->ws + L.xs.off, 0, L.xs.bytes, h->st));
  HIPCHK(h, hipMemsetAsync(h->ws + L.ys.off, 0, L.ys.bytes, h->st));
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  return CPD_OK;
}

template <typename T>
cpd_status prepare_impl(cpd_ctx* h, const double* U_import, const double* lam_import,
                        const double* omega) {
  const Layout& L = h->L;
  const auto t0 = std::chrono::steady_clock::now();
  if (h->p.method == CPD_METHOD_ORIGINAL) {
    if (U_import || lam_import || omega)
      return fail(h, CPD_E_ARG, "the original method takes no eigen-prep arguments");
    orig_prepare<T>(h->Xgram<T>(), h->p.M, h->p.beta, h->ws, L.orig, h->st);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(h->st));
    h->stage = Stage::Prepared;
    h->t_eig = 0.0;
    return CPD_OK;
  }
  if (h->p.eig_mode == CPD_EIG_IMPORT) {
    if (!U_import || !lam_import) return fail(h, CPD_E_ARG, "IMPORT needs U_import and lam_import");
    if (omega) return fail(h, CPD_E_ARG, "omega is only used by TOPK");
    import_eig_launch<T>(U_import, lam_import, h->at<T>(L.U), h->at<double>(L.lam),
                         h->at<double>(L.U64), h->p.M, h->p.K, h->st, h->permX());
    h->K = h->p.K;
  } else {
    if (U_import || lam_import) return fail(h, CPD_E_ARG, "U_import/lam_import are for IMPORT only");
    if (omega && h->p.eig_mode != CPD_EIG_TOPK) return fail(h, CPD_E_ARG, "omega is for TOPK only");
    EigRun r{};
    r.X = reinterpret_cast<const void*>(h->Xgram<T>());
    r.x_is_double = sizeof(T) == 8;
    r.M = h->p.M;
    r.beta = h->p.beta;
    r.mode = h->p.eig_mode;
    r.K = h->p.K;
    r.oversample = h->p.oversample;
    r.power_iters = h->p.power_iters;
    r.seed = h->p.seed;
    r.omega = omega;
    EigLayout slot_layout;
    char* eig_ws = h->ws;
    const EigLayout* el = &L.eig;
    double* U64 = h->at<double>(L.U64);
    if (L.eig_shared) {
      if (!h->eig_slot) return fail(h, CPD_E_STATE, "batch member prepared outside its batch");
      slot_layout = eig_layout(h->p.M, h->p.eig_mode, h->p.K, h->p.oversample,
                               eig_slot_u64_bytes(h->p));
      eig_ws = h->eig_slot;
      el = &slot_layout;
      U64 = reinterpret_cast<double*>(h->eig_slot);
    }
    if (omega && h->permX()) {  // rows into internal order, in the solver's own buffer
      double* om = reinterpret_cast<double*>(eig_ws + el->omega);
      gather_rows_launch<double>(omega, om, h->permX(), h->p.M, el->n, h->st);
      r.omega = om;
    }
    r.ws = eig_ws;
    r.L = el;
    r.U64 = U64;
    r.lam = h->at<double>(L.lam);
    r.Kcap = L.Kcap;
    r.st = h->st;
    r.jb = h->jb;
    int K = 0;
    std::string msg;
    const int rc = eig_prepare_run(r, &K, &msg);
    if (rc != 0 && rc != 4)
      return fail(h, rc == 1 ? CPD_E_NUMERIC : (rc == 3 ? CPD_E_UNSUPPORTED : CPD_E_DEVICE), msg);
    h->K = K;
    convert_u_launch<T>(U64, h->at<T>(L.U), (size_t)h->p.M * K, h->st);
    if (rc == 4) {  // usable, but truncated: reported, not hidden
      HIPCHK(h, hipGetLastError());
      HIPCHK(h, hipStreamSynchronize(h->st));
      h->t_eig = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      h->stage = Stage::Prepared;
      fail(h, CPD_NOT_CONVERGED, msg);
      return CPD_NOT_CONVERGED;
    }
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  h->t_eig = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  h->stage = Stage::Prepared;
  return CPD_OK;
}

template <typename T>
cpd_status estep_impl(cpd_ctx* h, void* logd, void* P1, void* Yt, void* tbar) {
  const Layout& L = h->L;
  if (h->permX()) {
    enqueue_estep<T>(h, 0, logd ? h->at<T>(L.logdtmp) : nullptr);
    if (logd) scatter_rows_launch<T>(h->at<T>(L.logdtmp), static_cast<T*>(logd), h->permY(), h->p.N, 1, h->st);
    if (P1) scatter_rows_launch<T>(h->at<T>(L.P1), static_cast<T*>(P1), h->permX(), h->p.M, 1, h->st);
    if (tbar) scatter_rows_launch<T>(h->at<T>(L.tbar), static_cast<T*>(tbar), h->permX(), h->p.M, 1, h->st);
  } else {
    enqueue_estep<T>(h, 0, static_cast<T*>(logd));
    if (P1) HIPCHK(h, hipMemcpyAsync(P1, h->ws + L.P1.off, sizeof(T) * h->p.M, hipMemcpyDeviceToDevice, h->st));
    if (tbar) HIPCHK(h, hipMemcpyAsync(tbar, h->ws + L.tbar.off, sizeof(T) * h->p.M, hipMemcpyDeviceToDevice, h->st));
  }
  if (Yt)
    unpack_launch<T>(h->at<P4<T>>(L.Yt), static_cast<T*>(Yt), h->p.M, h->p.D, h->st, h->permX(),
                     h->origin());
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  return CPD_OK;
}

__global__ void k_set_sigma2(DevScalars* sc, double s2) {
  if (threadIdx.x == 0) {
    sc->sigma2 = s2;
    sc->done = 0;
    sc->converged = 0;
    sc->nonfinite = 0;
    sc->chol_fail = 0;
  }
}

template <typename T>
cpd_status matches_impl(cpd_ctx* h, int mutual_only, int32_t* out) {
  const Layout& L = h->L;
  matches_launch<T>(h->at<P4<T>>(L.Xt), h->p.M, h->at<P4<T>>(L.Y), h->p.N, mutual_only,
                    h->permX(), h->permY(), h->at<int>(L.nnX), h->at<int>(L.nnY), out,
                    h->st);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  return CPD_OK;
}

template <typename T>
cpd_status solve_matches_impl(cpd_ctx* h, const int32_t* match, double sigma2, void* X_out,
                              void* W_out) {
  const Layout& L = h->L;
  hipLaunchKernelGGL(k_set_sigma2, dim3(1), dim3(64), 0, h->st, h->sc(), sigma2);
  match_in_launch<T>(match, h->p.M, h->p.N, h->permX(), h->invY(), h->at<P4<T>>(L.X),
                     h->at<P4<T>>(L.Y), h->at<T>(L.P1), h->at<P4<T>>(L.Yt), h->st);
  LowRankArgs<T> a{};
  a.X = h->at<P4<T>>(L.X);
  a.Yt = h->at<P4<T>>(L.Yt);
  a.P1 = h->at<T>(L.P1);
  a.U64 = h->at<double>(L.U64);
  a.lam = h->at<double>(L.lam);
  a.M = h->p.M;
  a.K = h->K;
  a.lmbda = h->p.lambda;
  a.sc = h->sc();
  a.gate = 0;
  a.ws = h->ws;
  a.L = &L.lr;
  a.Xnew = h->at<P4<T>>(L.Xnew);
  a.W = h->at<P4<T>>(L.W);
  lowrank_mstep_launch<T>(a, h->st);
  HIPCHK(h, hipMemcpyAsync(h->ws + L.Xt.off, h->ws + L.Xnew.off, L.Xt.bytes, hipMemcpyDeviceToDevice,
                           h->st));
  DevScalars s{};
  HIPCHK(h, hipMemcpyAsync(&s, h->sc(), sizeof(s), hipMemcpyDeviceToHost, h->st));
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  if (s.nonfinite) return fail(h, CPD_E_NUMERIC, "the matched system is not positive definite");
  if (X_out)
    unpack_launch<T>(h->at<P4<T>>(L.Xt), static_cast<T*>(X_out), h->p.M, h->p.D, h->st, h->permX(),
                     h->origin());
  if (W_out)
    unpack_launch<T>(h->at<P4<T>>(L.W), static_cast<T*>(W_out), h->p.M, h->p.D, h->st, h->permX());
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  return CPD_OK;
}

template <typename T>
cpd_status set_state_impl(cpd_ctx* h, const void* Xt, double sigma2) {
  const Layout& L = h->L;
  pack_launch<T>(static_cast<const T*>(Xt), h->at<P4<T>>(L.Xt), h->p.M, h->p.D, h->st, h->permX(),
                 h->origin());
  hipLaunchKernelGGL(k_set_sigma2, dim3(1), dim3(64), 0, h->st, h->sc(), sigma2);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  return CPD_OK;
}

template <typename T>
cpd_status get_state_impl(cpd_ctx* h, void* Xt, void* W, double* sigma2) {
  const Layout& L = h->L;
  if (Xt)
    unpack_launch<T>(h->at<P4<T>>(L.Xt), static_cast<T*>(Xt), h->p.M, h->p.D, h->st, h->permX(),
                     h->origin());
  if (W) unpack_launch<T>(h->at<P4<T>>(L.W), static_cast<T*>(W), h->p.M, h->p.D, h->st, h->permX());
  DevScalars s;
  HIPCHK(h, hipMemcpyAsync(&s, h->sc(), sizeof(s), hipMemcpyDeviceToHost, h->st));
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->st));
  if (sigma2) *sigma2 = s.sigma2;
  return CPD_OK;
}

template <typename T>
cpd_status time_impl(cpd_ctx* h, int reps, double* out) {
  EventGuard g[8];
  hipEvent_t e[8];
  for (int i = 0; i < 8; ++i) {
    HIPCHK(h, hipEventCreateWithFlags(&g[i].e, kTimingEventFlags));
    e[i] = g[i].e;
  }
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, h->st, h->sc(), 0);
  cpd_status s = CPD_OK;
  for (int r = 0; r < reps && s == CPD_OK; ++r) {
    (void)hipEventRecord(e[0], h->st);
    enqueue_estep<T>(h, 0, nullptr, &e[1]);  // e[1..5]
    enqueue_mstep<T>(h, 0);
    (void)hipEventRecord(e[6], h->st);
    enqueue_sigma2<T>(h, 0);
    (void)hipEventRecord(e[7], h->st);
    hipError_t err = hipEventSynchronize(e[7]);
    if (err != hipSuccess) {
      s = hip_fail(h, err, "hipEventSynchronize");
      break;
    }
    float ms[7];
    for (int i = 0; i < 7; ++i) (void)hipEventElapsedTime(&ms[i], e[i], e[i + 1]);
    float tot = 0;
    (void)hipEventElapsedTime(&tot, e[0], e[7]);
    acc[6] += ms[0];                // prescale
    acc[0] += ms[1];                // pass A
    acc[1] += ms[2];                // pass A merge + fix-up
    acc[2] += ms[3];                // pass B
    acc[3] += ms[4];                // pass B merge + fix-up
    acc[4] += ms[5];                // M-step
    acc[5] += ms[6];                // sigma^2
    acc[7] += tot;
  }
  if (s != CPD_OK) return s;
  for (int i = 0; i < 8; ++i) out[i] = acc[i] / reps;
  return CPD_OK;
}

bool is_f64(const cpd_ctx* h) { return h->p.precision == CPD_PREC_FP64; }

}  // namespace

extern "C" {

int32_t cpd_abi_version(void) { return CPD_ABI_VERSION; }

const char* cpd_build_info(void) { return "libfastcpd abi=1 target=gfx950"; }

const char* cpd_status_str(cpd_status s) {
  // a C caller may pass any int: read the bits as one, not as the enum
  int32_t v = 0;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case CPD_OK: return "CPD_OK";
    case CPD_NOT_CONVERGED: return "CPD_NOT_CONVERGED";
    case CPD_E_ARG: return "CPD_E_ARG";
    case CPD_E_STATE: return "CPD_E_STATE";
    case CPD_E_WORKSPACE: return "CPD_E_WORKSPACE";
    case CPD_E_DEVICE: return "CPD_E_DEVICE";
    case CPD_E_NUMERIC: return "CPD_E_NUMERIC";
    case CPD_E_UNSUPPORTED: return "CPD_E_UNSUPPORTED";
  }
  return "unknown status";
}

const char* cpd_last_error(cpd_handle h) { return h ? h->err.c_str() : g_last_error.c_str(); }

cpd_status cpd_workspace_size(const cpd_params* p, size_t* bytes) {
  if (!bytes) return fail(nullptr, CPD_E_ARG, "bytes is NULL");
  const cpd_status v = validate(p);
  if (v != CPD_OK) return v;
  *bytes = layout_for(*p).total;
  return CPD_OK;
}

cpd_status cpd_init(cpd_handle* out, const cpd_params* p, const void* X, const void* Y,
                    void* workspace, size_t workspace_bytes, void* hip_stream) {
  if (!out) return fail(nullptr, CPD_E_ARG, "handle pointer is NULL");
  *out = nullptr;
  const cpd_status v = validate(p);
  if (v != CPD_OK) return v;
  if (!X || !Y) return fail(nullptr, CPD_E_ARG, "X and Y must be device pointers");
  const Layout L = layout_for(*p);
  if (!workspace) return fail(nullptr, CPD_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(nullptr, CPD_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (workspace_bytes < L.total) return fail(nullptr, CPD_E_WORKSPACE, "workspace too small");
  const cpd_status d = check_device(nullptr);
  if (d != CPD_OK) return d;
  cpd_ctx* h = new (std::nothrow) cpd_ctx();
  if (!h) return fail(nullptr, CPD_E_DEVICE, "out of host memory");
  h->p = *p;
  h->L = L;
  if (p->precision == CPD_PREC_BF16X)  // fit pass B's splits to this device
    bfx_splits(p->M, p->N, bfx_resident_blocksB(), &h->L.splitsA, &h->L.chunkA, &h->L.splitsB,
               &h->L.chunkB);
  h->ws = static_cast<char*>(workspace);
  h->st = static_cast<hipStream_t>(hip_stream);
  const cpd_status s = is_f64(h) ? init_impl<double>(h, X, Y) : init_impl<float>(h, X, Y);
  if (s != CPD_OK) {
    g_last_error = h->err;
    delete h;
    return s;
  }
  *out = h;
  return CPD_OK;
}

cpd_status cpd_eig_prepare(cpd_handle h, const double* U_import, const double* lam_import,
                           const double* omega) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  return is_f64(h) ? prepare_impl<double>(h, U_import, lam_import, omega)
                   : prepare_impl<float>(h, U_import, lam_import, omega);
}

cpd_status cpd_eig_count(cpd_handle h, int32_t* K_out) {
  if (!h || !K_out) return fail(h, CPD_E_ARG, "NULL argument");
  if (h->stage != Stage::Prepared || h->p.method == CPD_METHOD_ORIGINAL)
    return fail(h, CPD_E_STATE, "no eigenpairs prepared");
  *K_out = h->K;
  return CPD_OK;
}

cpd_status cpd_eig_export(cpd_handle h, double* U_out, double* lam_out) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  if (h->stage != Stage::Prepared || h->p.method == CPD_METHOD_ORIGINAL)
    return fail(h, CPD_E_STATE, "no eigenpairs prepared");
  if (!U_out && !lam_out) return fail(h, CPD_E_ARG, "nothing to export");
  if (U_out && h->permX())
    scatter_rows_launch<double>(h->at<double>(h->L.U64), U_out, h->permX(), h->p.M, h->K, h->st);
  else if (U_out)
    HIPCHK(h, hipMemcpyAsync(U_out, h->ws + h->L.U64.off, sizeof(double) * (size_t)h->p.M * h->K,
                             hipMemcpyDeviceToDevice, h->st));
  if (lam_out)
    HIPCHK(h, hipMemcpyAsync(lam_out, h->ws + h->L.lam.off, sizeof(double) * h->K,
                             hipMemcpyDeviceToDevice, h->st));
  HIPCHK(h, hipStreamSynchronize(h->st));
  return CPD_OK;
}

cpd_status cpd_step(cpd_handle h, cpd_step_info* info) {
  const cpd_status r = ready_for_steps(h);
  if (r != CPD_OK) return r;
  return is_f64(h) ? step_impl<double>(h, info) : step_impl<float>(h, info);
}

cpd_status cpd_register(cpd_handle h, const void* W0, void* X_out, void* W_out, cpd_result* res) {
  const cpd_status r = ready_for_steps(h);
  if (r != CPD_OK) return r;
  return is_f64(h) ? register_impl<double>(h, W0, X_out, W_out, res)
                   : register_impl<float>(h, W0, X_out, W_out, res);
}

cpd_status cpd_set_state(cpd_handle h, const void* Xt, double sigma2) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  if (!Xt) return fail(h, CPD_E_ARG, "Xt is NULL");
  if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return fail(h, CPD_E_ARG, "sigma2 must be > 0");
  return is_f64(h) ? set_state_impl<double>(h, Xt, sigma2) : set_state_impl<float>(h, Xt, sigma2);
}

cpd_status cpd_get_state(cpd_handle h, void* Xt_out, void* W_out, double* sigma2_out) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  return is_f64(h) ? get_state_impl<double>(h, Xt_out, W_out, sigma2_out)
                   : get_state_impl<float>(h, Xt_out, W_out, sigma2_out);
}

cpd_status cpd_estep(cpd_handle h, void* logd, void* P1, void* Yt, void* tbar) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  return is_f64(h) ? estep_impl<double>(h, logd, P1, Yt, tbar)
                   : estep_impl<float>(h, logd, P1, Yt, tbar);
}

cpd_status cpd_matches(cpd_handle h, int32_t mutual_only, int32_t* match_out) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  if (!match_out) return fail(h, CPD_E_ARG, "match_out is NULL");
  return is_f64(h) ? matches_impl<double>(h, mutual_only != 0, match_out)
                   : matches_impl<float>(h, mutual_only != 0, match_out);
}

cpd_status cpd_solve_matches(cpd_handle h, const int32_t* match, double sigma2, void* X_out,
                             void* W_out) {
  if (!h) return fail(nullptr, CPD_E_ARG, "handle is NULL");
  if (!match) return fail(h, CPD_E_ARG, "match is NULL");
  if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return fail(h, CPD_E_ARG, "sigma2 must be > 0");
  if (h->stage != Stage::Prepared || h->p.method == CPD_METHOD_ORIGINAL)
    return fail(h, CPD_E_STATE, "cpd_solve_matches needs a prepared FAST or CPD-L handle");
  return is_f64(h) ? solve_matches_impl<double>(h, match, sigma2, X_out, W_out)
                   : solve_matches_impl<float>(h, match, sigma2, X_out, W_out);
}

cpd_status cpd_time_kernels(cpd_handle h, int32_t reps, double* out_ms) {
  const cpd_status r = ready_for_steps(h);
  if (r != CPD_OK) return r;
  if (reps < 1 || !out_ms) return fail(h, CPD_E_ARG, "reps must be >= 1 and out_ms non-NULL");
  return is_f64(h) ? time_impl<double>(h, reps, out_ms) : time_impl<float>(h, reps, out_ms);
}

// ---------------------------------------------------------------- batched
}  // extern "C"

namespace {
constexpr int kBatchChunks[] = {1024, 2048, 512, 4096};  // split-length candidates
constexpr int kBatchTiles[] = {4, 2};  // E-step points per thread (tiles of 256 x this)
constexpr int kBatchCands = 8;         // chunk-major: candidate c = kBatchChunks[c / 2], kBatchTiles[c % 2]
constexpr int kBatchSmallestChunk = 512;
// host threads (one stream each) that run the instances' eigen-preps in
// waves; their Jacobi solves are grouped into shared launches
constexpr int kPrepThreads = 32;

struct BatchHeader {
  size_t desc = 0, items = 0, done = 0, jac = 0, jacflags = 0, eigslot = 0, end = 0;
  size_t item_cap = 0;
  size_t slot_bytes = 0;  // one prepare thread's eigen-prep slot
};

size_t batch_item_capacity(int B, const cpd_params* p) {
  // the largest item count of any candidate plan (the smallest split length)
  size_t n = 0;
  for (int i = 0; i < B; ++i) {
    const int M = p[i].M, N = p[i].N;
    const int c = kBatchSmallestChunk;
    const size_t sA = (M + c - 1) / c, sB = (N + c - 1) / c;
    const size_t tA = (N + 511) / 512, tB = (M + 511) / 512;  // the smallest tile
    n += (((M + 63) & ~63) + N + 255) / 256;         // prescale (model part in whole tiles)
    n += tA * sA + tB * sB;                          // colsum, rowsum
    n += (N + 255) / 256 + (M + 255) / 256;          // merges
    n += (size_t)((M + 127) / 128) * 8;              // tpart (chunks x k groups)
    n += (size_t)eig_topk_max_cols();                // tmerge
    n += (M + 63) / 64 + (M + 255) / 256 + 1;        // apply, sigpart, final
  }
  return n;
}

BatchHeader batch_header(int B, const cpd_params* p) {
  BatchHeader h;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) & ~(size_t)255;
    return o;
  };
  h.desc = take((size_t)B * sizeof(InstDesc));
  h.item_cap = batch_item_capacity(B, p);
  h.items = take(h.item_cap * sizeof(int4));
  h.done = take(256);
  h.jac = take((size_t)kPrepThreads * sizeof(JacMember));
  h.jacflags = take((size_t)kPrepThreads * sizeof(int));
  for (int i = 0; i < B; ++i) h.slot_bytes = std::max(h.slot_bytes, eig_slot_bytes(p[i]));
  h.slot_bytes = (h.slot_bytes + 255) & ~(size_t)255;
  h.eigslot = take((size_t)std::min(B, kPrepThreads) * h.slot_bytes);
  h.end = off;
  return h;
}

cpd_status validate_batch(int B, const cpd_params* p) {
  if (B < 1 || !p) return fail(nullptr, CPD_E_ARG, "B must be >= 1 and params non-NULL");
  for (int i = 0; i < B; ++i) {
    const cpd_status v = validate(&p[i]);
    if (v != CPD_OK) return v;
    if (p[i].method != CPD_METHOD_FAST || p[i].precision != CPD_PREC_FP32 || p[i].D != 3 ||
        p[i].eig_mode == CPD_EIG_IMPORT)
      return fail(nullptr, CPD_E_UNSUPPORTED,
                  "batched registration runs Fast CPD, FP32, D = 3, FULL or TOPK eigen-prep");
  }
  return CPD_OK;
}

}  // namespace

struct cpd_batch_ctx {
  int B = 0;
  std::vector<cpd_params> p;
  std::vector<cpd_ctx*> inst;
  std::vector<size_t> inst_off;
  std::vector<int64_t> x_off, y_off;
  BatchHeader hd;
  char* ws = nullptr;
  hipStream_t user_st = nullptr, st = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  BatchItems items{};
  int chunk = kBatchChunks[0];
  int nb = kBatchTiles[0];
  bool prepared = false;
  std::string err;
  double tune_ms[kBatchCands] = {};
  ~cpd_batch_ctx() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto* h : inst) delete h;
    if (st) (void)hipStreamDestroy(st);
  }
};

namespace {

cpd_status bfail(cpd_batch_ctx* b, cpd_status s, const std::string& m) {
  g_last_error = m;
  if (b) b->err = m;
  return s;
}

// Descriptors and work lists for split length `chunk`; uploads both.
cpd_status batch_build(cpd_batch_ctx* b, int chunk, int nb) {
  std::vector<InstDesc> d(b->B);
  std::vector<int4> pre, cs, cm, rs, rm, tp, tp4, tm, ap, ap4, sp, in;
  int maxK = 1, maxK4 = 1;
  for (int i = 0; i < b->B; ++i) {
    const int K = b->inst[i]->K;
    if (fast_mstep_vec4<float>(K))
      maxK4 = std::max(maxK4, K);
    else
      maxK = std::max(maxK, K);
  }
  const int kt = maxK <= 256 ? 1 : (maxK <= 512 ? 2 : 4);
  for (int i = 0; i < b->B; ++i) {
    cpd_ctx* h = b->inst[i];
    const Layout& L = h->L;
    InstDesc& D = d[i];
    D.X = h->at<P4<float>>(L.X);
    D.Xt = h->at<P4<float>>(L.Xt);
    D.Xnew = h->at<P4<float>>(L.Xnew);
    D.Y = h->at<P4<float>>(L.Y);
    D.W = h->at<P4<float>>(L.W);
    D.xs = h->at<P4<float>>(L.xs);
    D.ys = h->at<P4<float>>(L.ys);
    D.Yt = h->at<P4<float>>(L.Yt);
    D.P1 = h->at<float>(L.P1);
    D.tbar = h->at<float>(L.tbar);
    D.partA = h->at<float>(L.partA);
    D.partB = h->at<float>(L.partB);
    D.llpart = h->at<double>(L.llpart);
    D.sigpart = h->at<double>(L.sigpart);
    D.U = h->at<float>(L.U);
    D.lam = h->at<double>(L.lam);
    D.tpart = h->at<float>(L.tpart);
    D.GT = h->at<P4<float>>(L.GT);
    D.HT = h->at<P4<float>>(L.HT);
    D.boxX = L.cull ? h->at<P4<float>>(L.boxX) : nullptr;
    D.boxY = L.cull ? h->at<P4<float>>(L.boxY) : nullptr;
    D.sc = h->sc();
    D.M = h->p.M;
    D.N = h->p.N;
    D.K = h->K;
    chunk_plan(D.M, D.N, chunk, &D.splitsA, &D.chunkA, &D.splitsB, &D.chunkB);
    if (D.splitsA > L.splitsA || D.splitsB > L.splitsB)
      return bfail(b, CPD_E_WORKSPACE, "batch split plan exceeds the partial buffers");
    D.mrows = L.mrows;
    D.mchunks = L.mchunks;
    const bool vec4 = fast_mstep_vec4<float>(D.K);
    // the 16-byte-load apply writes one sigma^2 partial per 64 rows
    D.sigblocks = vec4 ? (D.M + 63) / 64 : sigma2_blocks<float>(D.M);
    D.llblocks = (D.N + 255) / 256;
    D.w = h->p.w;
    D.lmbda = h->p.lambda;
    // with boxes the model part is padded to whole 64-point tiles
    const int pre_thr = (D.boxX ? ((D.M + 63) & ~63) : D.M) + D.N;
    for (int x = 0; x < (pre_thr + 255) / 256; ++x) pre.push_back(make_int4(i, x, 0, 0));
    const int tile = 256 * nb;
    for (int t = 0; t < (D.N + tile - 1) / tile; ++t)
      for (int s = 0; s < D.splitsA; ++s) cs.push_back(make_int4(i, t, s, 0));
    for (int x = 0; x < (D.N + 255) / 256; ++x) cm.push_back(make_int4(i, x, 0, 0));
    for (int t = 0; t < (D.M + tile - 1) / tile; ++t)
      for (int s = 0; s < D.splitsB; ++s) rs.push_back(make_int4(i, t, s, 0));
    for (int x = 0; x < (D.M + 255) / 256; ++x) rm.push_back(make_int4(i, x, 0, 0));
    if (vec4) {
      for (int c = 0; c < D.mchunks; ++c) tp4.push_back(make_int4(i, c, 0, 0));
    } else {
      for (int c = 0; c < D.mchunks; ++c)
        for (int g = 0; g < (D.K + 256 * kt - 1) / (256 * kt); ++g) tp.push_back(make_int4(i, c, g, 0));
    }
    for (int k = 0; k < D.K; ++k) tm.push_back(make_int4(i, k, 0, 0));
    for (int x = 0; x < (D.M + 63) / 64; ++x) (vec4 ? ap4 : ap).push_back(make_int4(i, x, 0, 0));
    if (!vec4)
      for (int x = 0; x < D.sigblocks; ++x) sp.push_back(make_int4(i, x, 0, 0));
    in.push_back(make_int4(i, 0, 0, 0));
  }
  std::vector<int4> all;
  std::vector<const std::vector<int4>*> lists = {&pre, &cs, &cm, &rs, &rm, &tp, &tp4,
                                                 &tm, &ap, &ap4, &sp, &in};
  for (auto* l : lists) all.insert(all.end(), l->begin(), l->end());
  if (all.size() > b->hd.item_cap) return bfail(b, CPD_E_WORKSPACE, "batch work list too large");
  int4* dev = reinterpret_cast<int4*>(b->ws + b->hd.items);
  size_t o = 0;
  const int4** ptrs[] = {&b->items.prescale, &b->items.colsum, &b->items.colmerge,
                         &b->items.rowsum, &b->items.rowmerge, &b->items.tpart,
                         &b->items.tpart4, &b->items.tmerge, &b->items.apply,
                         &b->items.apply4, &b->items.sigpart, &b->items.inst};
  int* counts[] = {&b->items.n_prescale, &b->items.n_colsum, &b->items.n_colmerge,
                   &b->items.n_rowsum, &b->items.n_rowmerge, &b->items.n_tpart,
                   &b->items.n_tpart4, &b->items.n_tmerge, &b->items.n_apply,
                   &b->items.n_apply4, &b->items.n_sigpart, &b->items.n_inst};
  for (size_t q = 0; q < lists.size(); ++q) {
    *ptrs[q] = dev + o;
    *counts[q] = (int)lists[q]->size();
    o += lists[q]->size();
  }
  b->items.nb = nb;
  b->items.kt = kt;
  b->items.maxK = maxK;
  b->items.maxK4 = maxK4;
  b->items.done_count = reinterpret_cast<int*>(b->ws + b->hd.done);
  InstDesc* dd = reinterpret_cast<InstDesc*>(b->ws + b->hd.desc);
  HIPCHK(nullptr, hipMemcpyAsync(dd, d.data(), sizeof(InstDesc) * d.size(), hipMemcpyHostToDevice, b->st));
  HIPCHK(nullptr, hipMemcpyAsync(dev, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice, b->st));
  HIPCHK(nullptr, hipStreamSynchronize(b->st));
  b->chunk = chunk;
  b->nb = nb;
  return CPD_OK;
}

const InstDesc* batch_desc(const cpd_batch_ctx* b) {
  return reinterpret_cast<const InstDesc*>(b->ws + b->hd.desc);
}

__global__ void kb_reset(const InstDesc* __restrict__ d, int B, int restart) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  DevScalars* sc = d[i].sc;
  if (restart) {
    sc->sigma2 = sc->sigma2_start;
    sc->sigma2_floor = fmax(1e-10 * sc->sigma2_start, sc->floor_data);
    sc->dsigma2 = 0.0;
    sc->nonfinite = 0;
  }
  sc->iter = 0;
  sc->done = 0;
  sc->converged = 0;
}

// Back to the start state (Xt = X, sigma^2 = sigma^2_0) for every instance.
cpd_status batch_restart(cpd_batch_ctx* b) {
  for (int i = 0; i < b->B; ++i) {
    cpd_ctx* h = b->inst[i];
    HIPCHK(nullptr, hipMemcpyAsync(h->ws + h->L.Xt.off, h->ws + h->L.X.off, h->L.X.bytes,
                                   hipMemcpyDeviceToDevice, b->st));
  }
  hipLaunchKernelGGL(kb_reset, dim3((b->B + 255) / 256), dim3(256), 0, b->st, batch_desc(b), b->B, 1);
  HIPCHK(nullptr, hipGetLastError());
  return CPD_OK;
}

}  // namespace

extern "C" {

cpd_status cpd_batch_workspace_size(int32_t B, const cpd_params* p, size_t* bytes) {
  if (!bytes) return fail(nullptr, CPD_E_ARG, "bytes is NULL");
  const cpd_status v = validate_batch(B, p);
  if (v != CPD_OK) return v;
  size_t total = batch_header(B, p).end;
  for (int i = 0; i < B; ++i) total += (layout_for(p[i], kBatchSmallestChunk).total + 255) & ~(size_t)255;
  *bytes = total;
  return CPD_OK;
}

cpd_status cpd_batch_init(cpd_batch* out, int32_t B, const cpd_params* p, const float* X_packed,
                          const float* Y_packed, const int64_t* x_off, const int64_t* y_off,
                          void* workspace, size_t bytes, void* hip_stream) {
  if (!out) return fail(nullptr, CPD_E_ARG, "batch handle pointer is NULL");
  *out = nullptr;
  const cpd_status v = validate_batch(B, p);
  if (v != CPD_OK) return v;
  if (!X_packed || !Y_packed || !x_off || !y_off)
    return fail(nullptr, CPD_E_ARG, "packed points and offsets are required");
  for (int i = 0; i < B; ++i) {
    if (x_off[i + 1] - x_off[i] != p[i].M || y_off[i + 1] - y_off[i] != p[i].N || x_off[i] < 0 ||
        y_off[i] < 0)
      return fail(nullptr, CPD_E_ARG, "offsets do not match M and N of instance " + std::to_string(i));
  }
  size_t need = 0;
  const cpd_status sz = cpd_batch_workspace_size(B, p, &need);
  if (sz != CPD_OK) return sz;
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 || bytes < need)
    return fail(nullptr, CPD_E_WORKSPACE, "batch workspace missing, misaligned or too small");
  const cpd_status d = check_device(nullptr);
  if (d != CPD_OK) return d;
  auto* b = new (std::nothrow) cpd_batch_ctx();
  if (!b) return fail(nullptr, CPD_E_DEVICE, "out of host memory");
  b->B = B;
  b->p.assign(p, p + B);
  b->x_off.assign(x_off, x_off + B + 1);
  b->y_off.assign(y_off, y_off + B + 1);
  b->ws = static_cast<char*>(workspace);
  b->user_st = static_cast<hipStream_t>(hip_stream);
  b->hd = batch_header(B, p);
  hipError_t e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(nullptr, e, "hipStreamCreateWithFlags");
  }
  size_t off = b->hd.end;
  for (int i = 0; i < B; ++i) {
    auto* h = new (std::nothrow) cpd_ctx();
    if (!h) {
      delete b;
      return fail(nullptr, CPD_E_DEVICE, "out of host memory");
    }
    h->p = p[i];
    h->L = layout_for(p[i], kBatchSmallestChunk);
    h->ws = b->ws + off;
    h->st = b->st;
    b->inst.push_back(h);
    b->inst_off.push_back(off);
    off += (h->L.total + 255) & ~(size_t)255;
    const cpd_status s = init_impl<float>(h, X_packed + 3 * x_off[i], Y_packed + 3 * y_off[i]);
    if (s != CPD_OK) {
      const std::string m = h->err;
      delete b;
      return fail(nullptr, s, m);
    }
  }
  *out = b;
  return CPD_OK;
}

cpd_status cpd_batch_prepare(cpd_batch b, int32_t tune) {
  if (!b) return fail(nullptr, CPD_E_ARG, "batch handle is NULL");
  if (tune < 0 || tune > 1 + kBatchCands)
    return bfail(b, CPD_E_ARG, "tune must be 0, 1 or 2 + a candidate index (0..7)");
  // per-instance eigen-prep in waves of up to kPrepThreads host threads, one
  // stream each; the Jacobi solves of a wave run as grouped launches
  const int nt = std::min(kPrepThreads, b->B);
  std::vector<hipStream_t> sts(nt, nullptr);
  for (auto& s : sts) HIPCHK(nullptr, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  JacobiBatcher jb(reinterpret_cast<JacMember*>(b->ws + b->hd.jac),
                   reinterpret_cast<int*>(b->ws + b->hd.jacflags), kPrepThreads);
  std::vector<cpd_status> rc(b->B, CPD_OK);
  // instances whose FULL eigen-prep is the dense Jacobi on all M points go
  // first, widest first, so that they share waves (a wave's Jacobi launches
  // run as many steps as its widest solve needs)
  std::vector<int> order(b->B);
  for (int i = 0; i < b->B; ++i) order[i] = i;
  auto dense_n = [&](int i) {
    const cpd_params& q = b->p[i];
    return (q.eig_mode == CPD_EIG_FULL && eig_full_capacity(q.M) == q.M) ? q.M : 0;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return dense_n(a) > dense_n(c); });
  for (int w0 = 0; w0 < b->B; w0 += nt) {
    const int wn = std::min(nt, b->B - w0);
    jb.begin(wn);
    std::vector<std::thread> th;
    for (int t = 0; t < wn; ++t) {
      th.emplace_back([&, t]() {
        const int i = order[w0 + t];
        cpd_ctx* h = b->inst[i];
        h->st = sts[t];
        h->jb = &jb;
        h->eig_slot = b->ws + b->hd.eigslot + (size_t)t * b->hd.slot_bytes;
        rc[i] = prepare_impl<float>(h, nullptr, nullptr, nullptr);
        jb.leave();
        h->eig_slot = nullptr;
        h->jb = nullptr;
        h->st = b->st;
        if (rc[i] == CPD_NOT_CONVERGED) rc[i] = CPD_OK;  // a truncated FULL basis is usable
      });
    }
    for (auto& x : th) x.join();
  }
  for (auto& s : sts) (void)hipStreamDestroy(s);
  for (int i = 0; i < b->B; ++i)
    if (rc[i] != CPD_OK) return bfail(b, rc[i], "instance " + std::to_string(i) + ": " + b->inst[i]->err);
  // pick the split length and the E-step tile: time two batched iterations
  // per candidate
  int best = kBatchChunks[0], best_nb = kBatchTiles[0];
  if (tune >= 2) {
    best = kBatchChunks[(tune - 2) / 2];
    best_nb = kBatchTiles[(tune - 2) % 2];
  } else if (tune == 1) {
    float best_ms = 1e30f;
    EventGuard g0, g1;
    HIPCHK(nullptr, hipEventCreate(&g0.e));
    HIPCHK(nullptr, hipEventCreate(&g1.e));
    hipEvent_t e0 = g0.e, e1 = g1.e;
    for (int c = 0; c < kBatchCands; ++c) {
      const int ch = kBatchChunks[c / 2], nb = kBatchTiles[c % 2];
      const cpd_status s = batch_build(b, ch, nb);
      if (s != CPD_OK) return s;
      hipLaunchKernelGGL(kb_reset, dim3((b->B + 255) / 256), dim3(256), 0, b->st, batch_desc(b), b->B, 0);
      batch_iteration_launch(batch_desc(b), b->items, b->st);  // warm
      (void)hipEventRecord(e0, b->st);
      for (int r = 0; r < 2; ++r) batch_iteration_launch(batch_desc(b), b->items, b->st);
      (void)hipEventRecord(e1, b->st);
      HIPCHK(nullptr, hipEventSynchronize(e1));
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      b->tune_ms[c] = ms / 2;
      if (ms < best_ms) {
        best_ms = ms;
        best = ch;
        best_nb = nb;
      }
    }
  }
  cpd_status s = batch_build(b, best, best_nb);
  if (s != CPD_OK) return s;
  s = batch_restart(b);
  if (s != CPD_OK) return s;
  // capture one batched iteration (every stage, every instance) as a graph
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  HIPCHK(nullptr, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  batch_iteration_launch(batch_desc(b), b->items, b->st);
  HIPCHK(nullptr, hipStreamEndCapture(b->st, &b->graph));
  HIPCHK(nullptr, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  HIPCHK(nullptr, hipStreamSynchronize(b->st));
  b->prepared = true;
  return CPD_OK;
}

cpd_status cpd_batch_register(cpd_batch b, const float* W0_packed, const double* sigma2_start,
                              float* X_out_packed, cpd_result* res) {
  if (!b) return fail(nullptr, CPD_E_ARG, "batch handle is NULL");
  if (!b->prepared) return bfail(b, CPD_E_STATE, "cpd_batch_prepare must run first");
  if (sigma2_start)
    for (int i = 0; i < b->B; ++i)
      if (!std::isfinite(sigma2_start[i]))
        return bfail(b, CPD_E_ARG, "sigma2_start entries must be finite");
  // order after the caller's stream; every event is released on every return
  EventGuard g0, g1, gt0, gt1;
  HIPCHK(nullptr, hipEventCreate(&g0.e));
  HIPCHK(nullptr, hipEventCreate(&g1.e));
  HIPCHK(nullptr, hipEventCreate(&gt0.e));
  HIPCHK(nullptr, hipEventCreate(&gt1.e));
  hipEvent_t ev0 = g0.e, ev1 = g1.e, t0 = gt0.e, t1 = gt1.e;
  (void)hipEventRecord(ev0, b->user_st);
  HIPCHK(nullptr, hipStreamWaitEvent(b->st, ev0, 0));
  const cpd_status rs = batch_restart(b);
  if (rs != CPD_OK) return rs;
  for (int i = 0; i < b->B; ++i) {
    cpd_ctx* h = b->inst[i];
    if (W0_packed) {
      const float* w0 = W0_packed + 3 * b->x_off[i];
      if (h->permX()) {  // into the instance's internal order (Xnew is free here)
        float* tmp = h->at<float>(h->L.Xnew);
        gather_rows_launch<float>(w0, tmp, h->permX(), h->p.M, 3, b->st);
        w0 = tmp;
      }
      phi_apply_launch<float>(h->at<P4<float>>(h->L.X), w0, h->at<P4<float>>(h->L.Xt), h->p.M, 3,
                              h->p.beta, b->st);
    }
    if (sigma2_start && sigma2_start[i] > 0.0)
      reset_sigma2_launch<float>(h->at<P4<float>>(h->L.Xt), h->at<P4<float>>(h->L.Y), h->p.M,
                                 h->p.N, 3, h->sc(), h->at<double>(h->L.initpart), b->st,
                                 kS2Given, sigma2_start[i]);
    else if (W0_packed && !(h->p.sigma2_init > 0.0))
      reset_sigma2_launch<float>(h->at<P4<float>>(h->L.Xt), h->at<P4<float>>(h->L.Y), h->p.M,
                                 h->p.N, 3, h->sc(), h->at<double>(h->L.initpart), b->st,
                                 kS2Warm);
  }
  HIPCHK(nullptr, hipGetLastError());
  int max_iter = 1;
  for (auto& q : b->p) max_iter = std::max(max_iter, q.max_iter);
  (void)hipEventRecord(t0, b->st);
  int done = 0, iters = 0;
  while (iters < max_iter && done < b->B) {
    const int r = std::min(8, max_iter - iters);
    for (int k = 0; k < r; ++k) HIPCHK(nullptr, hipGraphLaunch(b->exec, b->st));
    iters += r;
    HIPCHK(nullptr, hipMemcpyAsync(&done, b->items.done_count, sizeof(int), hipMemcpyDeviceToHost, b->st));
    HIPCHK(nullptr, hipStreamSynchronize(b->st));
  }
  (void)hipEventRecord(t1, b->st);
  HIPCHK(nullptr, hipEventSynchronize(t1));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, t0, t1);
  std::vector<DevScalars> s(b->B);
  for (int i = 0; i < b->B; ++i) {
    cpd_ctx* h = b->inst[i];
    HIPCHK(nullptr, hipMemcpyAsync(&s[i], h->sc(), sizeof(DevScalars), hipMemcpyDeviceToHost, b->st));
    if (X_out_packed)
      unpack_launch<float>(h->at<P4<float>>(h->L.Xt), X_out_packed + 3 * b->x_off[i], h->p.M, 3,
                           b->st, h->permX(), h->origin());
  }
  HIPCHK(nullptr, hipGetLastError());
  (void)hipEventRecord(ev1, b->st);
  HIPCHK(nullptr, hipStreamWaitEvent(b->user_st, ev1, 0));
  HIPCHK(nullptr, hipStreamSynchronize(b->st));
  bool all = true, bad = false;
  for (int i = 0; i < b->B; ++i) {
    if (res) {
      res[i].iters = s[i].iter;
      res[i].converged = s[i].converged;
      res[i].sigma2 = s[i].sigma2;
      res[i].t_c = 0.0;
      res[i].t_iter = 0.0;
      res[i].t_eig = b->inst[i]->t_eig;
      res[i].t_o = ms * 1e-3;  // the whole batched run
    }
    all = all && s[i].converged;
    bad = bad || s[i].nonfinite;
  }
  if (bad) return bfail(b, CPD_E_NUMERIC, "an instance's sigma^2 became non-finite");
  return all ? CPD_OK : CPD_NOT_CONVERGED;
}

cpd_status cpd_batch_info(cpd_batch b, int32_t* chunk, int32_t* tile, double* tune_ms,
                          int32_t* K) {
  if (!b) return fail(nullptr, CPD_E_ARG, "batch handle is NULL");
  if (chunk) *chunk = b->chunk;
  if (tile) *tile = 256 * b->nb;
  if (tune_ms)
    for (int c = 0; c < kBatchCands; ++c) tune_ms[c] = b->tune_ms[c];
  if (K)
    for (int i = 0; i < b->B; ++i) K[i] = b->inst[i]->K;
  return CPD_OK;
}

cpd_status cpd_batch_destroy(cpd_batch b) {
  delete b;
  return CPD_OK;
}

// ---------------------------------------------------------------- network
cpd_status cpdnet_param_count(size_t* count) {
  if (!count) return fail(nullptr, CPD_E_ARG, "count is NULL");
  *count = net_offsets().count;
  return CPD_OK;
}

cpd_status cpdnet_init(float* params, uint64_t seed, float out_scale, void* stream) {
  if (!params) return fail(nullptr, CPD_E_ARG, "params is NULL");
  const cpd_status d = check_device(nullptr);
  if (d != CPD_OK) return d;
  net_init_launch(params, seed, out_scale, static_cast<hipStream_t>(stream));
  HIPCHK(nullptr, hipGetLastError());
  return CPD_OK;
}

static cpd_status net_dims(int32_t batch, int32_t M, int32_t N, int32_t precision) {
  if (batch < 1 || M < 1 || N < 1 || (int64_t)batch * std::max(M, N) > (1 << 24))
    return fail(nullptr, CPD_E_ARG, "batch, M, N must be >= 1 with batch * max(M, N) <= 2^24");
  if (precision != CPDNET_BF16 && precision != CPDNET_FP32)
    return fail(nullptr, CPD_E_ARG, "network precision must be CPDNET_BF16 or CPDNET_FP32");
  return CPD_OK;
}

cpd_status cpdnet_workspace_size(int32_t batch, int32_t M, int32_t N, int32_t precision,
                                 size_t* bytes) {
  if (!bytes) return fail(nullptr, CPD_E_ARG, "bytes is NULL");
  const cpd_status v = net_dims(batch, M, N, precision);
  if (v != CPD_OK) return v;
  *bytes = net_ws_layout(batch, M, N, precision).end;
  return CPD_OK;
}

cpd_status cpdnet_forward(const float* params, const float* X, const float* Y, int32_t batch,
                          int32_t M, int32_t N, int32_t precision, float* W0_out, void* ws,
                          size_t bytes, void* stream) {
  const cpd_status v = net_dims(batch, M, N, precision);
  if (v != CPD_OK) return v;
  if (!params || !X || !Y || !W0_out) return fail(nullptr, CPD_E_ARG, "NULL array");
  const NetWs L = net_ws_layout(batch, M, N, precision);
  if (!ws || bytes < L.end || reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(nullptr, CPD_E_WORKSPACE, "network workspace missing, misaligned or too small");
  const cpd_status d = check_device(nullptr);
  if (d != CPD_OK) return d;
  hipStream_t st = static_cast<hipStream_t>(stream);
  net_forward_launch(params, X, Y, batch, M, N, W0_out, static_cast<char*>(ws), L, precision, st);
  HIPCHK(nullptr, hipGetLastError());
  return CPD_OK;
}

}  // extern "C"

// Library-owned device scratch for cpdnet_forward_noalloc, one copy per device
// (it lives as long as the process).  In host code this name is only a
// stand-in: kernels and copies get the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
cpd_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(nullptr, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, CPD_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHK(nullptr, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(nullptr, CPD_E_DEVICE, "no device address for the static scratch");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return CPD_OK;
}
}  // namespace

extern "C" {

cpd_status cpdnet_forward_noalloc(const float* params, const float* X, const float* Y,
                                  int32_t batch, int32_t M, int32_t N, int32_t precision,
                                  float* W0_out, void* stream) {
  const cpd_status v = net_dims(batch, M, N, precision);
  if (v != CPD_OK) return v;
  if (!params || !X || !Y || !W0_out) return fail(nullptr, CPD_E_ARG, "NULL array");
  const NetWs L = net_ws_layout(batch, M, N, precision);
  if (L.end > kNoAllocScratchBytes)
    return fail(nullptr, CPD_E_WORKSPACE,
                "batch, M, N need " + std::to_string(L.end) + " bytes of network workspace; "
                "the static scratch holds " + std::to_string(kNoAllocScratchBytes));
  const cpd_status d = check_device(nullptr);
  if (d != CPD_OK) return d;
  void* ws = nullptr;
  const cpd_status a = scratch_address(&ws);
  if (a != CPD_OK) return a;
  net_forward_launch(params, X, Y, batch, M, N, W0_out, static_cast<char*>(ws), L, precision,
                     static_cast<hipStream_t>(stream));
  HIPCHK(nullptr, hipGetLastError());
  return CPD_OK;
}

cpd_status cpdnet_loss_grad(const float* params, const float* X, const float* Y, const float* V,
                            int32_t batch, int32_t M, int32_t N, int32_t precision, double beta,
                            float* grad_out, double* loss_out, void* ws, size_t bytes,
                            void* stream) {
  const cpd_status v = net_dims(batch, M, N, precision);
  if (v != CPD_OK) return v;
  if (!params || !X || !Y || !V || !grad_out) return fail(nullptr, CPD_E_ARG, "NULL array");
  if (!(beta > 0.0)) return fail(nullptr, CPD_E_ARG, "beta must be > 0");
  const NetWs L = net_ws_layout(batch, M, N, precision);
  if (!ws || bytes < L.end || reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(nullptr, CPD_E_WORKSPACE, "network workspace missing, misaligned or too small");
  const cpd_status d = check_device(nullptr);
  if (d != CPD_OK) return d;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  double* ldev = reinterpret_cast<double*>(w + L.loss);
  net_loss_grad_launch(params, X, Y, V, batch, M, N, beta, grad_out, ldev, w, L, precision, st);
  HIPCHK(nullptr, hipGetLastError());
  if (loss_out) {
    HIPCHK(nullptr, hipMemcpyAsync(loss_out, ldev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(nullptr, hipStreamSynchronize(st));
  }
  return CPD_OK;
}

cpd_status cpdnet_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                       float lr, void* stream) {
  if (!params || !m || !v || !grad || step < 1 || !(lr > 0.f))
    return fail(nullptr, CPD_E_ARG, "bad Adam arguments");
  net_adam_launch(params, m, v, grad, step, lr, static_cast<hipStream_t>(stream));
  HIPCHK(nullptr, hipGetLastError());
  return CPD_OK;
}

cpd_status cpdnet_synth(float* X, float* Y, float* V, float* Wsc, int32_t batch, int32_t M,
                        int32_t shape, double beta, double coef, double jitter,
                        double outlier_frac, uint64_t seed0, void* stream) {
  const cpd_status vd = net_dims(batch, M, M, CPDNET_BF16);
  if (vd != CPD_OK) return vd;
  if (!X || !Y || !V || !Wsc || !(beta > 0.0) || !(outlier_frac >= 0.0 && outlier_frac <= 1.0) ||
      (shape != CPDNET_SHAPE_SPHERE && shape != CPDNET_SHAPE_BUMPS))
    return fail(nullptr, CPD_E_ARG, "bad synth arguments");
  net_synth_launch(X, Y, V, Wsc, batch, M, shape, beta, coef, jitter, outlier_frac, seed0,
                   static_cast<hipStream_t>(stream));
  HIPCHK(nullptr, hipGetLastError());
  return CPD_OK;
}

cpd_status cpd_destroy(cpd_handle h) {
  delete h;
  return CPD_OK;
}

}  // extern "C"
