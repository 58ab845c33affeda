// C ABI of librtgevc.so: argument checks, workspace carve-up and the launch
// sequence of the blocked robust solver (Algorithm 1 of Section 3 with the
// robustness of Section 4 and the task types of Section 5):
//   pre-processing  ->  for each tile row r from the bottom:
//                          solve row r   (tips for tile r, diagonal solves for tiles j > r)
//                          update rows above from row r (every tile column j >= r at once)
//                   ->  post-processing (consolidation / normalisation).
// All work is enqueued on the caller's stream; nothing is allocated, nothing waits.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "rtgevc.h"
#include "back.hpp"
#include "complex.hpp"
#include "layout.hpp"
#include "schedule.hpp"
#include "slices.hpp"

namespace rgev {
void launch_preprocess(const PencilDesc& P, hipStream_t s);
void launch_solve(const PencilDesc& P, int r, hipStream_t s);
hipError_t launch_band_chain(const PencilDesc& P, int r_lo, int r_hi, hipStream_t s);
bool launch_update(const PencilDesc& P, int k_lo, int k_hi, int j_lo, int s_lo, int s_hi, hipStream_t s);
void launch_consolidate(const PencilDesc& P, hipStream_t s);
void launch_preprocess_batched(const PencilDesc* D, int n, int64_t max_m, int max_tiles, hipStream_t s);
void launch_solve_batched(const PencilDesc* D, int n, int mb, int max_tiles, int R, int t, int io, hipStream_t s);
void launch_update_batched(const PencilDesc* D, int n, int mb, int max_tiles, int R, int t, int part, int a, int c,
                           int kmax, hipStream_t s);
void launch_consolidate_batched(const PencilDesc* D, int n, int64_t max_m, hipStream_t s);
void launch_eigvals_out(const PencilDesc& P, double* are, double* aim, double* bet, hipStream_t s);
void launch_backtransform(const BackDesc& B, hipStream_t s);
void launch_left_flip(int64_t m, const double* A, int64_t lda, double* B, hipStream_t s);
void launch_left_select(int64_t m, const int32_t* sel, int32_t* out, hipStream_t s);
void launch_left_finish(int64_t m, const int8_t* blkp, double* Y, int64_t ldy, int32_t* scales, hipStream_t s);
hipError_t launch_walk(const PencilDesc& P, const WalkDesc& W, hipStream_t s);
void launch_refine_setup(const PencilDesc& P, const RefineDesc& R, hipStream_t s);
void launch_refine_estimate(const PencilDesc& P, const RefineDesc& R, int pass, bool final_pass, hipStream_t s);
void launch_refine_residual(const PencilDesc& P, const RefineDesc& R, hipStream_t s);
void launch_refine_apply(const PencilDesc& P, const RefineDesc& R, hipStream_t s);
void launch_complex_realify(const ComplexDesc& C, hipStream_t s);
void launch_complex_extract(const ComplexDesc& C, hipStream_t s);
}  // namespace rgev

using namespace rgev;

namespace {

constexpr size_t kAlign = 256;
__host__ __device__ inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct TuneSingle {
  int64_t m_max;
  int32_t mb, band, schedule, split;   // FP64
  int32_t mb_mixed, band_mixed, split_mixed; // mixed precision (always the band wavefront)
};
struct TuneBatch {
  int64_t m_max;
  int32_t mb;
};
#include "tuning_table.inc"

const TuneSingle& tune_single(int64_t m) {
  const int n = (int)(sizeof(kTuneSingle) / sizeof(kTuneSingle[0]));
  for (int i = 0; i < n - 1; ++i)
    if (m <= kTuneSingle[i].m_max) return kTuneSingle[i];
  return kTuneSingle[n - 1];
}

bool mixed(const rtgevc_opts* o) { return o && o->precision == 1; }
int resolve_band(int64_t m, const rtgevc_opts* o) {
  if (o && o->band) return o->band;
  return mixed(o) ? tune_single(m).band_mixed : tune_single(m).band;
}
int resolve_schedule(int64_t m, const rtgevc_opts* o);

int resolve_mb(int64_t m, const rtgevc_opts* o) {
  if (o && o->mb) return o->mb;
  return mixed(o) ? tune_single(m).mb_mixed : tune_single(m).mb;
}

// tiles per launch of the band schedule's updates of the rows above a band, 0 for one
// launch (automatic: the table entry of m when the tile size and band are the table's as
// well, else one launch)
int resolve_split(int64_t m, const rtgevc_opts* o) {
  if (o && o->split != 0) return o->split > 0 ? o->split : 0;
  const TuneSingle& t = tune_single(m);
  const bool mx = mixed(o);
  if (resolve_mb(m, o) != (mx ? t.mb_mixed : t.mb) || resolve_band(m, o) != (mx ? t.band_mixed : t.band)) return 0;
  return mx ? t.split_mixed : t.split;
}

// C(b) of the band schedule as one launch (band_chain_kernel) for FP64 tile updates and bands
// of more than one row; the mixed mode keeps its in-band updates on the int8 kernel
bool use_chain(const PencilDesc& P) { return P.precision == 0 && P.band > 1; }

bool opts_ok(const rtgevc_opts* o) {
  if (!o) return true;
  if (o->mb != 0 && o->mb != 32 && o->mb != 64 && o->mb != 128) return false;
  if (o->normalize != 0 && o->normalize != 1) return false;
  if (o->band < 0 || o->band > kMaxBand) return false;
  if (o->schedule < 0 || o->schedule > 2) return false;
  if (o->watchdog < 0) return false;
  if (o->precision < 0 || o->precision > 1) return false;
  if (o->precision == 1 && o->schedule == 2) return false;   // the walker runs FP64 updates
  if (o->max_refine < -1 || o->max_refine > 3) return false;
  if (o->refine_bits < 0 || o->refine_bits > 100) return false;
  if (o->split < -1) return false;
  if (o->grid < 0) return false;
  return true;
}

// refinement sweeps of a call: mixed precision only; max_refine 0 = 1, -1 = none
int resolve_sweeps(const rtgevc_opts* o) {
  if (!o || o->precision != 1) return 0;
  if (o->max_refine < 0) return 0;
  return o->max_refine == 0 ? 1 : o->max_refine;
}

// flag threshold: 2^-refine_bits, or by default the residual bound 64 m 2^-53
double resolve_tau(int64_t m, const rtgevc_opts* o) {
  if (o && o->refine_bits > 0) return ldexp(1.0, -o->refine_bits);
  return 64.0 * (double)m * 1.1102230246251565e-16;
}

int resolve_precision(const rtgevc_opts* o) { return (o && o->precision == 1) ? 1 : 0; }

// 1 = band wavefront on two streams, 2 = persistent walker (FP64 updates only)
int resolve_schedule(int64_t m, const rtgevc_opts* o) {
  if (o && o->schedule) return o->schedule;
  if (o && o->precision == 1) return 1;
  return tune_single(m).schedule;
}
constexpr int kDefaultSpinLimit = 1 << 26;   // about two seconds of waiting

struct Carve {
  size_t off = 0;
  template <class T>
  __host__ __device__ T* take(char* base, size_t count) {
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += up(count * sizeof(T));
    return p;
  }
};

// Lays out the workspace; with base == nullptr it only measures.  W keeps 2 band source
// rows (band wavefront) or, with walk != nullptr, every source row (persistent walker).
__host__ __device__ size_t carve(PencilDesc& P, char* base, int64_t m, int mb, int band, WalkDesc* walk = nullptr,
                                 int precision = 0, RefineDesc* ref = nullptr) {
  const int Mmax = tile_bound(m, mb);
  const int wslots = walk ? Mmax : 2 * band;
  Carve c;
  P.ctrl = c.take<Ctrl>(base, 1);
  P.blk = c.take<int8_t>(base, m);
  P.sel = c.take<int8_t>(base, m);
  P.tileof = c.take<int32_t>(base, m);
  P.edges = c.take<int32_t>(base, Mmax + 1);
  P.ar = c.take<double>(base, m);
  P.ai = c.take<double>(base, m);
  P.be = c.take<double>(base, m);
  P.cnS = c.take<double>(base, m);
  P.cnT = c.take<double>(base, m);
  P.nu = c.take<double>(base, (size_t)Mmax * Mmax);
  P.exps = c.take<int32_t>(base, (size_t)Mmax * m);
  P.norms = c.take<double>(base, (size_t)Mmax * m);
  P.segn = c.take<double>(base, (size_t)Mmax * m);
  P.W = c.take<double>(base, (size_t)wslots * Mmax * w_tile_doubles(mb));
  P.eW = c.take<int32_t>(base, (size_t)wslots * m);
  P.nW = c.take<double>(base, (size_t)wslots * m);
  P.mb = mb;
  P.Mmax = Mmax;
  P.band = band;
  P.wslots = wslots;
  P.precision = precision;
  if (precision == 1) {
    const size_t pairs = (size_t)Mmax * (Mmax - 1) / 2;
    P.Aslc = c.take<int4>(base, pairs * kSlices * slice_packets(mb));
    P.Aexp = c.take<int32_t>(base, pairs * mb);
    P.Wslc = c.take<int4>(base, (size_t)wslots * Mmax * kSlices * slice_packets(mb));
    P.Wexp = c.take<int32_t>(base, (size_t)wslots * m);
    P.stmax = c.take<unsigned long long>(base, (size_t)2 * Mmax);
    P.exps_next = c.take<int32_t>(base, (size_t)Mmax * m);
    P.norms_next = c.take<unsigned long long>(base, (size_t)Mmax * m);
  }
  if (ref) {
    ref->G = c.take<double>(base, (size_t)m * kSketch);
    ref->GS = c.take<double>(base, (size_t)m * kSketch);
    ref->GT = c.take<double>(base, (size_t)m * kSketch);
    ref->cS = c.take<double>(base, m);
    ref->cT = c.take<double>(base, m);
    ref->PS = c.take<double>(base, (size_t)m * kSketch);
    ref->PT = c.take<double>(base, (size_t)m * kSketch);
    ref->dS = c.take<double>(base, m);
    ref->dT = c.take<double>(base, m);
    ref->zexp = c.take<int32_t>(base, m);
    ref->rf = c.take<int8_t>(base, m);
    ref->fits = c.take<int8_t>(base, m);
    ref->tflag = c.take<int32_t>(base, Mmax);
    ref->part = c.take<double>(base, (size_t)((m + 1023) / 1024) * m * (2 * kSketch + 2));
    ref->Zc = c.take<double>(base, (size_t)m * m);
    ref->cexps = c.take<int32_t>(base, (size_t)Mmax * m);
    ref->cnorms = c.take<double>(base, (size_t)Mmax * m);
  }
  if (walk) {
    walk->cnt = c.take<int32_t>(base, (size_t)Mmax * Mmax);
    walk->solved = c.take<int32_t>(base, (size_t)Mmax * Mmax);
    walk->levels = c.take<int64_t>(base, (size_t)2 * Mmax + 1);
    walk->next = c.take<int32_t>(base, 1);
    walk->tickets = c.take<int4>(base, (size_t)walk_tasks(Mmax));
  }
  return c.off;
}

int hip_code(hipError_t e) { return e == hipSuccess ? 0 : -1000 - (int)e; }

// ---- batches ----
// Pencils are grouped by tile size; each group runs in lock-step over bands of R tile rows
// (the single-pencil band schedule without the look-ahead): step t takes band B_p - 1 - t
// of every pencil p of the group (B_p bands from the top, the last one possibly short),
// solves its rows bottom-up, each followed by the in-band update of the band rows above
// it, then applies the band to every row above it; one launch carries the same part of a
// step for the whole group.  The descriptor table lives at the
// start of the workspace and is written by small set-up kernels whose arguments carry
// the per-pencil parameters by value, so the whole call is a fixed sequence of kernel
// launches (a HIP graph can capture and replay it).

struct BatchArg {
  int64_t m, lds, ldt, ldz, off;
  const double* S;
  const double* T;
  double* Z;
  int32_t* scales;
  const int32_t* select;
  int32_t* info;
  int32_t mb, normalize, band;
};
constexpr int kSetupPerLaunch = 32;   // 32 x 104 bytes of kernel arguments per launch
struct BatchSetup {
  BatchArg a[kSetupPerLaunch];
  int32_t n, first;
};
static_assert(sizeof(BatchSetup) <= 4096, "kernel arguments of one set-up launch");

__global__ void batch_setup_kernel(BatchSetup su, PencilDesc* table, char* work) {
  const int i = threadIdx.x;
  if (i >= su.n) return;
  const BatchArg& a = su.a[i];
  PencilDesc P = {};
  P.m = a.m;
  P.lds = a.lds;
  P.ldt = a.ldt;
  P.ldz = a.ldz;
  P.S = a.S;
  P.T = a.T;
  P.Z = a.Z;
  P.scales = a.scales;
  P.select = a.select;
  carve(P, work + a.off, a.m, a.mb, a.band);
  P.info = a.info ? a.info : &P.ctrl->info_local;
  P.normalize = a.normalize;
  table[su.first + i] = P;
}

constexpr int kBatchMbs[3] = {32, 64, 128};
constexpr int kBatchBand = 3;   // tile rows per band of a batch's lock-step (opts->band overrides)

// tiles per launch of a batch step's update of the rows above the next band, summed over
// the group's pencils (opts->split overrides; 0 = one launch per step)
constexpr int kBatchSplit = 0;

int batch_band(const rtgevc_opts* o) { return (o && o->band) ? o->band : kBatchBand; }

int batch_split(const rtgevc_opts* o) {
  const int v = o ? o->split : 0;
  return v > 0 ? v : (v < 0 ? 0 : kBatchSplit);
}

int batch_mb(int64_t m, const rtgevc_opts* o) {
  if (o && o->mb) return o->mb;
  const int n = (int)(sizeof(kTuneBatch) / sizeof(kTuneBatch[0]));
  for (int i = 0; i < n - 1; ++i)
    if (m <= kTuneBatch[i].m_max) return kTuneBatch[i].mb;
  return kTuneBatch[n - 1].mb;
}

// Workspace of a batch: the descriptor table, then each non-empty pencil's own area.
size_t batch_layout(int32_t count, const int64_t* m, const rtgevc_opts* o, int64_t* offs) {
  size_t off = up((size_t)(count > 0 ? count : 0) * sizeof(PencilDesc));
  for (int i = 0; i < count; ++i) {
    if (offs) offs[i] = (int64_t)off;
    if (m[i] <= 0) continue;
    PencilDesc P;
    memset(&P, 0, sizeof(P));
    off += carve(P, nullptr, m[i], batch_mb(m[i], o), batch_band(o));
  }
  return off;
}

// Per-device side stream and events for the look-ahead schedule, created once (default
// priority) and kept until the process ends.  The enqueue of one call holds g_aux_mu, so
// calls from several host threads do not interleave their event records.
struct Aux {
  hipStream_t side = nullptr;
  hipEvent_t evC = nullptr, evJ = nullptr, evU[2] = {nullptr, nullptr};
  bool ok = false;
};
std::mutex g_aux_mu;
Aux g_aux[64];

hipError_t get_aux(Aux** out) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  Aux& a = g_aux[dev];
  if (!a.ok) {
    err = hipStreamCreateWithFlags(&a.side, hipStreamNonBlocking);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&a.evC, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&a.evJ, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&a.evU[0], hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventCreateWithFlags(&a.evU[1], hipEventDisableTiming);
    if (err != hipSuccess) return err;
    a.ok = true;
  }
  *out = &a;
  return hipSuccess;
}

// The blocked back-substitution for tile rows [0, rows): the band wavefront schedule
// (schedule.hpp) enqueued on the caller's stream sa and the side stream.  mark(kind,
// before, stream, range) brackets each launch (kind 1 = solve, 2 = update with its range
// {k_lo, k_hi, j_lo, s_lo, s_hi}, nullptr for a solve); rows at or beyond the device's tile
// count M are no-ops in the kernels.
template <class Mark>
hipError_t enqueue_rows(const PencilDesc& P, int rows, hipStream_t sa, Aux& ax, Mark&& mark) {
  hipError_t err = hipSuccess;
  struct Ops {
    const PencilDesc& P;
    hipStream_t st[2];
    hipEvent_t ev[4];
    Mark& mark;
    hipError_t& err;
    bool ok(hipError_t e) {
      if (err == hipSuccess) err = e;
      return err == hipSuccess;
    }
    bool solve(int i, int s) {
      mark(1, true, st[s], nullptr);
      launch_solve(P, i, st[s]);
      mark(1, false, st[s], nullptr);
      return err == hipSuccess;
    }
    bool update(int k_lo, int k_hi, int j_lo, int s_lo, int s_hi, int s) {
      const int rng[5] = {k_lo, k_hi, j_lo, s_lo, s_hi};
      mark(2, true, st[s], rng);
      launch_update(P, k_lo, k_hi, j_lo, s_lo, s_hi, st[s]);
      mark(2, false, st[s], rng);
      return err == hipSuccess;
    }
    bool chain(int r_lo, int r_hi, int s) {
      if (!use_chain(P)) return chain_steps(r_lo, r_hi, s, *this);
      mark(1, true, st[s], nullptr);   // (timed as a solve launch: it holds the band's solves)
      ok(launch_band_chain(P, r_lo, r_hi, st[s]));
      mark(1, false, st[s], nullptr);
      return err == hipSuccess;
    }
    bool record(int e, int s) { return ok(hipEventRecord(ev[e], st[s])); }
    bool wait(int s, int e) { return ok(hipStreamWaitEvent(st[s], ev[e], 0)); }
  } ops{P, {sa, ax.side}, {ax.evC, ax.evJ, ax.evU[0], ax.evU[1]}, mark, err};
  band_schedule(rows, P.band, P.split, ops);
  return err;
}

// Events of the timed entry point, created once per device and reused by later calls
// (held until the process ends).
std::mutex g_event_mu;
std::vector<hipEvent_t> g_events[64];

hipError_t get_events(int n, hipEvent_t** out) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::vector<hipEvent_t>& v = g_events[dev];
  while ((int)v.size() < n) {
    hipEvent_t e;
    err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    v.push_back(e);
  }
  *out = v.data();
  return hipSuccess;
}

int check_common(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt, void* work,
                 size_t work_bytes, const rtgevc_opts* opts, int i_work, int i_bytes, int i_opts) {
  if (m < 0) return -1;
  if (m > 0 && !S) return -2;
  if (lds < (m > 1 ? m : 1)) return -3;
  if (m > 0 && !T) return -4;
  if (ldt < (m > 1 ? m : 1)) return -5;
  if (!opts_ok(opts)) return -i_opts;
  if (m > 0) {
    if (!work || (reinterpret_cast<uintptr_t>(work) % kAlign) != 0) return -i_work;
    if (work_bytes < rtgevc_workspace_size(m, opts)) return -i_bytes;
  }
  return 0;
}

PencilDesc make_desc(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt,
                     const int32_t* select, double* Z, int64_t ldz, int32_t* scales, int32_t* info,
                     void* work, const rtgevc_opts* opts, WalkDesc* walk = nullptr, RefineDesc* ref = nullptr) {
  PencilDesc P;
  memset(&P, 0, sizeof(P));
  P.m = m;
  P.lds = lds;
  P.ldt = ldt;
  P.ldz = ldz;
  P.S = S;
  P.T = T;
  P.Z = Z;
  P.scales = scales;
  P.select = select;
  carve(P, static_cast<char*>(work), m, resolve_mb(m, opts), resolve_band(m, opts), walk, resolve_precision(opts),
        resolve_sweeps(opts) > 0 ? ref : nullptr);
  if (ref) ref->tau = resolve_tau(m, opts);
  P.split = resolve_split(m, opts);
  P.info = info ? info : &P.ctrl->info_local;
  P.normalize = opts ? opts->normalize : 1;
  if (walk) {
    walk->spin_limit = (opts && opts->watchdog > 0) ? opts->watchdog : kDefaultSpinLimit;
    walk->grid = opts ? opts->grid : 0;
  }
  return P;
}

// tile size of the back-transformation: 64 or 128 (opts->mb; 0 or 32: 128 from m = 2048)
int back_mb(int64_t m, const rtgevc_opts* o) {
  if (o && (o->mb == 64 || o->mb == 128)) return o->mb;
  return m >= 2048 ? 128 : 64;
}

// workspace of the back-transformation (base == nullptr: size only)
size_t back_carve(BackDesc& B, char* base, int64_t m, int mb) {
  const int nt = (int)((m + mb - 1) / mb);
  Carve c;
  B.blk = c.take<int8_t>(base, m);
  B.zmax = c.take<double>(base, m);
  B.vmax = c.take<unsigned long long>(base, 1);
  B.info_local = c.take<int32_t>(base, 1);
  B.Zp = c.take<double>(base, (size_t)back_tile_offset(mb, nt));
  B.mb = mb;
  B.nt = nt;
  return c.off;
}

// The band schedule with every launch on one stream (no side stream, no events): the same
// launches in the same order as the two-stream look-ahead, so the same eigenvectors.
hipError_t enqueue_rows_one_stream(const PencilDesc& P, int rows, hipStream_t s) {
  struct Ops {
    const PencilDesc& P;
    hipStream_t s;
    bool solve(int i, int) {
      launch_solve(P, i, s);
      return true;
    }
    bool update(int k_lo, int k_hi, int j_lo, int s_lo, int s_hi, int) {
      launch_update(P, k_lo, k_hi, j_lo, s_lo, s_hi, s);
      return true;
    }
    bool chain(int r_lo, int r_hi, int st) {
      if (!use_chain(P)) return chain_steps(r_lo, r_hi, st, *this);
      err = launch_band_chain(P, r_lo, r_hi, s);
      return err == hipSuccess;
    }
    bool record(int, int) { return true; }
    bool wait(int, int) { return true; }
    hipError_t err = hipSuccess;   // the chain launch's set-up error, if any
  } ops{P, s};
  band_schedule(rows, P.band, 0, ops);   // (one stream: no other launches to let in)
  const hipError_t e = hipGetLastError();
  return ops.err != hipSuccess ? ops.err : e;
}

// Refinement sweeps of a mixed-precision result (refine.hip): estimate and flag, FP64
// residual of the flagged columns, correction solve through the blocked solver in
// correction mode (rows(C) enqueues it), z <- z - d; a last estimate reports the columns
// still above the threshold (info bit 64).
template <class Rows>
hipError_t enqueue_refine(const PencilDesc& P, const RefineDesc& R, int sweeps, hipStream_t s, Rows&& rows) {
  launch_refine_setup(P, R, s);
  PencilDesc C = P;
  C.Z = R.Zc;
  C.ldz = P.m;
  C.exps = R.cexps;
  C.norms = R.cnorms;
  C.segn = nullptr;   // (the correction's segment maxima are not needed; z's stay)
  C.sel = R.rf;
  C.rhs = 1;
  C.tflag = R.tflag;
  C.scales = nullptr;
  hipError_t err = hipSuccess;
  for (int sw = 0; sw < sweeps && err == hipSuccess; ++sw) {
    launch_refine_estimate(P, R, sw, false, s);
    launch_refine_residual(P, R, s);
    err = rows(C);
    launch_refine_apply(P, R, s);
  }
  launch_refine_estimate(P, R, sweeps, true, s);
  return err == hipSuccess ? hipGetLastError() : err;
}

// The right-eigenvector path (rtgevc after its argument checks); *out gets the pencil
// descriptor (its block structure stays valid in the workspace).  one_stream: the band
// schedule without the side stream (no stream or event is created).
hipError_t enqueue_right(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt,
                         const int32_t* select, double* Z, int64_t ldz, int32_t* scales, int32_t* info,
                         void* work, const rtgevc_opts* opts, hipStream_t s, PencilDesc* out,
                         bool one_stream = false, int cform = 0) {
  if (resolve_schedule(m, opts) == 2) {
    WalkDesc W;
    PencilDesc P = make_desc(m, S, lds, T, ldt, select, Z, ldz, scales, info, work, opts, &W);
    P.cform = cform;
    *out = P;
    launch_preprocess(P, s);
    hipError_t err = launch_walk(P, W, s);
    launch_consolidate(P, s);
    return err == hipSuccess ? hipGetLastError() : err;
  }
  RefineDesc R;
  PencilDesc P = make_desc(m, S, lds, T, ldt, select, Z, ldz, scales, info, work, opts, nullptr, &R);
  P.cform = cform;
  *out = P;
  const int sweeps = resolve_sweeps(opts);
  if (one_stream) {
    launch_preprocess(P, s);
    hipError_t err = enqueue_rows_one_stream(P, P.Mmax, s);
    if (err == hipSuccess && sweeps > 0)
      err = enqueue_refine(P, R, sweeps, s, [&](const PencilDesc& C) { return enqueue_rows_one_stream(C, C.Mmax, s); });
    launch_consolidate(P, s);
    return err == hipSuccess ? hipGetLastError() : err;
  }
  std::lock_guard<std::mutex> lock(g_aux_mu);
  Aux* ax = nullptr;
  hipError_t err = get_aux(&ax);
  if (err != hipSuccess) return err;
  launch_preprocess(P, s);
  err = enqueue_rows(P, P.Mmax, s, *ax, [](int, bool, hipStream_t, const int*) {});
  if (err == hipSuccess && sweeps > 0)
    err = enqueue_refine(P, R, sweeps, s, [&](const PencilDesc& C) {
      return enqueue_rows(C, C.Mmax, s, *ax, [](int, bool, hipStream_t, const int*) {});
    });
  launch_consolidate(P, s);
  return err == hipSuccess ? hipGetLastError() : err;
}

// ---- the entry point that allocates nothing ----
// Its workspace is this file-scope device array instead of a caller's buffer.  Host code
// never passes the array's name to a kernel (on the host the name is only a stand-in):
// the device address is looked up once per device with hipGetSymbolAddress and kept.
static __device__ __align__(256) char scratch[RTGEVC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64];

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return err;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}


// workspace of the left solve beyond the right solve's: S', T' (m^2 doubles each), select'
size_t left_extra_bytes(int64_t m) {
  return up((size_t)(2 * m * m) * sizeof(double) + (size_t)m * sizeof(int32_t));
}

}  // namespace

extern "C" {

size_t rtgevc_workspace_size(int64_t m, const rtgevc_opts* opts) {
  if (m < 0) return 0;
  if (m == 0) return kAlign;
  PencilDesc P;
  memset(&P, 0, sizeof(P));
  WalkDesc W;
  RefineDesc R;
  return carve(P, nullptr, m, resolve_mb(m, opts), resolve_band(m, opts),
               resolve_schedule(m, opts) == 2 ? &W : nullptr, resolve_precision(opts),
               resolve_sweeps(opts) > 0 ? &R : nullptr);
}

int rtgevc(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt, const int32_t* select,
           double* Z, int64_t ldz, int32_t* scales, int32_t* info, void* work, size_t work_bytes,
           const rtgevc_opts* opts, void* stream) {
  int rc = check_common(m, S, lds, T, ldt, work, work_bytes, opts, 11, 12, 13);
  if (rc) return rc;
  if (m > 0 && !Z) return -7;
  if (ldz < (m > 1 ? m : 1)) return -8;
  if (m == 0) return 0;
  PencilDesc P;
  return hip_code(enqueue_right(m, S, lds, T, ldt, select, Z, ldz, scales, info, work, opts,
                                static_cast<hipStream_t>(stream), &P));
}

int rtgevc_noalloc(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt,
                   const int32_t* select, double* Z, int64_t ldz, int32_t* scales, int32_t* info,
                   const rtgevc_opts* opts, void* stream) {
  if (m < 0) return -1;
  if (m > 0 && !S) return -2;
  if (lds < (m > 1 ? m : 1)) return -3;
  if (m > 0 && !T) return -4;
  if (ldt < (m > 1 ? m : 1)) return -5;
  if (m > 0 && !Z) return -7;
  if (ldz < (m > 1 ? m : 1)) return -8;
  if (!opts_ok(opts)) return -11;
  if (m == 0) return 0;
  if (rtgevc_workspace_size(m, opts) > (size_t)RTGEVC_NOALLOC_SCRATCH_BYTES) return RTGEVC_ERR_SCRATCH;
  void* work = nullptr;
  hipError_t err = scratch_address(&work);
  if (err != hipSuccess) return hip_code(err);
  PencilDesc P;
  return hip_code(enqueue_right(m, S, lds, T, ldt, select, Z, ldz, scales, info, work, opts,
                                static_cast<hipStream_t>(stream), &P, /*one_stream=*/true));
}

size_t rtgevc_complex_workspace_size(int64_t m, const rtgevc_opts* opts) {
  if (m < 0) return 0;
  if (m == 0) return kAlign;
  const size_t n2 = (size_t)(2 * m) * (size_t)(2 * m);
  return rtgevc_workspace_size(2 * m, opts) + 3 * up(n2 * sizeof(double)) + 2 * up((size_t)(2 * m) * sizeof(int32_t));
}

int rtgevc_complex(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt, const int32_t* select,
                   double* Z, int64_t ldz, int32_t* scales, int32_t* info, void* work, size_t work_bytes,
                   const rtgevc_opts* opts, void* stream) {
  const int64_t lo = m > 1 ? m : 1;
  if (m < 0) return -1;
  if (m > 0 && !S) return -2;
  if (lds < lo) return -3;
  if (m > 0 && !T) return -4;
  if (ldt < lo) return -5;
  if (m > 0 && !Z) return -7;
  if (ldz < lo) return -8;
  if (!opts_ok(opts)) return -13;
  if (m == 0) return 0;
  if (!work || (reinterpret_cast<uintptr_t>(work) % kAlign) != 0) return -11;
  if (work_bytes < rtgevc_complex_workspace_size(m, opts)) return -12;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t m2 = 2 * m;
  const size_t n2 = (size_t)m2 * (size_t)m2;
  // [the real path's workspace for order 2m][S2][T2][Z2][sel2][scales2]
  char* base = static_cast<char*>(work);
  size_t off = rtgevc_workspace_size(m2, opts);
  ComplexDesc C;
  memset(&C, 0, sizeof(C));
  C.m = m;
  C.lds = lds;
  C.ldt = ldt;
  C.ldz = ldz;
  C.S = S;
  C.T = T;
  C.Z = Z;
  C.scales = scales;
  C.select = select;
  C.S2 = reinterpret_cast<double*>(base + off);
  off += up(n2 * sizeof(double));
  C.T2 = reinterpret_cast<double*>(base + off);
  off += up(n2 * sizeof(double));
  C.Z2 = reinterpret_cast<double*>(base + off);
  off += up(n2 * sizeof(double));
  C.sel2 = reinterpret_cast<int32_t*>(base + off);
  off += up((size_t)m2 * sizeof(int32_t));
  C.scales2 = reinterpret_cast<int32_t*>(base + off);
  C.normalize = opts ? opts->normalize : 1;
  launch_complex_realify(C, s);
  PencilDesc P;
  hipError_t err = enqueue_right(m2, C.S2, m2, C.T2, m2, C.sel2, C.Z2, m2, C.scales2, info, work, opts, s, &P,
                                 false, /*cform=*/1);
  launch_complex_extract(C, s);
  if (err == hipSuccess) err = hipGetLastError();
  return hip_code(err);
}

size_t rtgevc_left_workspace_size(int64_t m, const rtgevc_opts* opts) {
  if (m < 0) return 0;
  if (m == 0) return kAlign;
  return rtgevc_workspace_size(m, opts) + left_extra_bytes(m);
}

int rtgevc_left(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt, const int32_t* select,
                double* Y, int64_t ldy, int32_t* scales, int32_t* info, void* work, size_t work_bytes,
                const rtgevc_opts* opts, void* stream) {
  int rc = check_common(m, S, lds, T, ldt, work, work_bytes, opts, 11, 12, 13);
  if (rc) return rc;
  if (m > 0 && !Y) return -7;
  if (ldy < (m > 1 ? m : 1)) return -8;
  if (m == 0) return 0;
  if (work_bytes < rtgevc_left_workspace_size(m, opts)) return -12;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // (S', T', select') after the right solve's own workspace
  char* extra = static_cast<char*>(work) + rtgevc_workspace_size(m, opts);
  double* Sp = reinterpret_cast<double*>(extra);
  double* Tp = Sp + m * m;
  int32_t* selp = reinterpret_cast<int32_t*>(Tp + m * m);
  launch_left_flip(m, S, lds, Sp, s);
  launch_left_flip(m, T, ldt, Tp, s);
  if (select) launch_left_select(m, select, selp, s);
  PencilDesc P;
  hipError_t err = enqueue_right(m, Sp, m, Tp, m, select ? selp : nullptr, Y, ldy, scales, info, work, opts, s, &P);
  launch_left_finish(m, P.blk, Y, ldy, scales, s);
  if (err == hipSuccess) err = hipGetLastError();
  return hip_code(err);
}

int rtgevc_eigvals(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt, double* alpha_re,
                   double* alpha_im, double* beta, int32_t* info, void* work, size_t work_bytes,
                   const rtgevc_opts* opts, void* stream) {
  int rc = check_common(m, S, lds, T, ldt, work, work_bytes, opts, 10, 11, 12);
  if (rc) return rc;
  if (m > 0 && !alpha_re) return -6;
  if (m > 0 && !alpha_im) return -7;
  if (m > 0 && !beta) return -8;
  if (m == 0) return 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PencilDesc P = make_desc(m, S, lds, T, ldt, nullptr, nullptr, m, nullptr, info, work, opts);
  launch_preprocess(P, s);
  launch_eigvals_out(P, alpha_re, alpha_im, beta, s);
  return hip_code(hipGetLastError());
}

size_t rtgevc_backtransform_workspace_size(int64_t m, const rtgevc_opts* opts) {
  if (m < 0) return 0;
  if (m == 0) return kAlign;
  BackDesc B;
  memset(&B, 0, sizeof(B));
  return back_carve(B, nullptr, m, back_mb(m, opts));
}

int rtgevc_backtransform(int64_t m, const double* S, int64_t lds, const double* V, int64_t ldv,
                         const double* Z, int64_t ldz, const int32_t* scales, double* X, int64_t ldx,
                         int32_t* xscales, int32_t* info, void* work, size_t work_bytes,
                         const rtgevc_opts* opts, void* stream) {
  const int64_t lo = m > 1 ? m : 1;
  if (m < 0) return -1;
  if (m > 0 && !S) return -2;
  if (lds < lo) return -3;
  if (m > 0 && !V) return -4;
  if (ldv < lo) return -5;
  if (m > 0 && !Z) return -6;
  if (ldz < lo) return -7;
  if (m > 0 && !X) return -9;
  if (ldx < lo) return -10;
  if (m > 0 && !xscales) return -11;
  if (!opts_ok(opts)) return -15;
  if (m == 0) return 0;
  if (!work || (reinterpret_cast<uintptr_t>(work) % kAlign) != 0) return -13;
  if (work_bytes < rtgevc_backtransform_workspace_size(m, opts)) return -14;
  if (X != Z && X == V) return -9;   // X may be Z, never V
  if (X == Z && ldx != ldz) return -10;
  BackDesc B;
  memset(&B, 0, sizeof(B));
  B.m = m;
  B.S = S;
  B.lds = lds;
  B.V = V;
  B.ldv = ldv;
  B.Z = Z;
  B.ldz = ldz;
  B.scales = scales;
  B.X = X;
  B.ldx = ldx;
  B.xscales = xscales;
  back_carve(B, static_cast<char*>(work), m, back_mb(m, opts));
  B.info = info ? info : B.info_local;
  B.normalize = opts ? opts->normalize : 1;
  launch_backtransform(B, static_cast<hipStream_t>(stream));
  return hip_code(hipGetLastError());
}

int rtgevc_timed(int64_t m, const double* S, int64_t lds, const double* T, int64_t ldt, const int32_t* select,
                 double* Z, int64_t ldz, int32_t* scales, int32_t* info, void* work, size_t work_bytes,
                 const rtgevc_opts* opts, void* stream, double* stats, int nstats) {
  int rc = check_common(m, S, lds, T, ldt, work, work_bytes, opts, 11, 12, 13);
  if (rc) return rc;
  if (m > 0 && !Z) return -7;
  if (ldz < (m > 1 ? m : 1)) return -8;
  if (!stats || nstats < RTGEVC_TIMED_NSTATS) return -15;
  for (int i = 0; i < nstats; ++i) stats[i] = 0.0;
  if (m == 0) return 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool walker = resolve_schedule(m, opts) == 2;
  WalkDesc W;
  RefineDesc R;
  PencilDesc P = make_desc(m, S, lds, T, ldt, select, Z, ldz, scales, info, work, opts, walker ? &W : nullptr,
                           walker ? nullptr : &R);
  const int sweeps = walker ? 0 : resolve_sweeps(opts);
  // events bracket every launch on the stream it runs on: the schedule's launches for the
  // largest tile count (a dry run of the same schedule), plus the few outside it
  struct Count {
    bool fused;
    int n = 0;
    bool solve(int, int) { ++n; return true; }
    bool update(int, int, int, int, int, int) { ++n; return true; }
    bool chain(int r_lo, int r_hi, int s) {
      if (!fused) return chain_steps(r_lo, r_hi, s, *this);
      ++n;
      return true;
    }
    bool record(int, int) { return true; }
    bool wait(int, int) { return true; }
  } cnt{use_chain(P)};
  band_schedule(P.Mmax, P.band, P.split, cnt);
  const int nlaunch = cnt.n + 8;
  const int nev = 2 * nlaunch;
  std::lock_guard<std::mutex> lock(g_event_mu);
  std::lock_guard<std::mutex> lock2(g_aux_mu);
  hipEvent_t* ev = nullptr;
  int used = 0;
  hipError_t err = get_events(nev, &ev);
  if (err != hipSuccess) return hip_code(err);
  Aux* ax = nullptr;
  err = get_aux(&ax);
  if (err != hipSuccess) return hip_code(err);
  auto mark_on = [&](hipStream_t st) {
    if (used >= nev) {   // (not reached: the count above bounds the launches)
      if (err == hipSuccess) err = hipErrorInvalidValue;
      return;
    }
    const hipError_t e = hipEventRecord(ev[used++], st);
    if (err == hipSuccess) err = e;
  };
  auto mark = [&]() { mark_on(s); };
  struct Span { int cls, e0, e1, side; int rng[5]; };
  Span* spans = new Span[nlaunch];
  int nsp = 0;
  mark();
  launch_preprocess(P, s);
  mark();
  spans[nsp++] = Span{0, 0, 1, 0, {}};
  int32_t M = 0;
  err = hipMemcpyAsync(&M, &P.ctrl->M, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  if (err == hipSuccess && walker) {
    // the whole task graph is one launch (counted with the updates)
    const int e0 = used;
    mark();
    err = launch_walk(P, W, s);
    mark();
    spans[nsp++] = Span{2, e0, e0 + 1, 0, {}};
  } else if (err == hipSuccess) {
    const hipError_t e = enqueue_rows(P, M, s, *ax, [&](int kind, bool before, hipStream_t st, const int* rng) {
      mark_on(st);
      if (!before && nsp < nlaunch) {
        spans[nsp] = Span{kind, used - 2, used - 1, st == ax->side ? 1 : 0, {}};
        if (rng)
          for (int q = 0; q < 5; ++q) spans[nsp].rng[q] = rng[q];
        ++nsp;
      }
    });
    if (err == hipSuccess) err = e;
  }
  if (err == hipSuccess && sweeps > 0) {
    // the refinement is one span (its correction solves' launches are not marked)
    const int f0 = used;
    mark();
    err = enqueue_refine(P, R, sweeps, s, [&](const PencilDesc& C) {
      return enqueue_rows(C, M, s, *ax, [](int, bool, hipStream_t, const int*) {});
    });
    mark();
    spans[nsp++] = Span{4, f0, f0 + 1, 0, {}};
  }
  const int c0 = used;
  mark();
  launch_consolidate(P, s);
  mark();
  spans[nsp++] = Span{3, c0, c0 + 1, 0, {}};
  if (err == hipSuccess) err = hipGetLastError();
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  int32_t* edges = new int32_t[M + 1];
  if (err == hipSuccess && M > 0) err = hipMemcpy(edges, P.edges, sizeof(int32_t) * (M + 1), hipMemcpyDeviceToHost);
  if (err == hipSuccess) {
    float ms = 0.0f;
    err = hipEventElapsedTime(&ms, ev[0], ev[used - 1]);
    stats[0] = ms;
    for (int i = 0; i < nsp && err == hipSuccess; ++i) {
      err = hipEventElapsedTime(&ms, ev[spans[i].e0], ev[spans[i].e1]);
      if (spans[i].cls == 4) {
        stats[12] += ms;
        continue;
      }
      stats[1 + spans[i].cls] += ms;
      stats[5 + spans[i].cls] += 1.0;
      if (spans[i].cls == 2 && !walker) {
        // an update launch: algorithmic flops of its range (target rows [k_lo, k_hi), columns
        // j >= j_lo, sources s_lo .. min(s_hi, j)); the side stream's launches also apart
        const int* g = spans[i].rng;
        const int k1 = g[1] < M ? g[1] : M, s1 = g[4] < M - 1 ? g[4] : M - 1;
        double fl = 0.0;
        if (g[0] < k1)
          for (int r = g[3]; r <= s1; ++r) {
            const int j0 = g[2] > r ? g[2] : r;
            fl += 4.0 * (double)(edges[k1] - edges[g[0]]) * (edges[r + 1] - edges[r]) * (edges[M] - edges[j0]);
          }
        stats[9] += fl;
        if (spans[i].side) {
          stats[14] += ms;
          stats[15] += fl;
          stats[16] += 1.0;
        }
      }
    }
    stats[13] = sweeps;
    if (walker) {
      // algorithmic flops of the tile updates: sum over k < r <= j of 2 h_k (2 h_r) h_j
      double fl = 0.0;
      for (int r = M - 1; r >= 1; --r) {
        const double hr = edges[r + 1] - edges[r];
        const double hj_sum = (double)(edges[M] - edges[r]);   // columns of tiles j >= r
        const double hk_sum = (double)edges[r];                // rows of tiles k < r
        fl += 4.0 * hk_sum * hr * hj_sum;
      }
      stats[9] = fl;
    }
    stats[10] = M;
    stats[11] = P.mb;
  }
  delete[] edges;
  delete[] spans;
  return hip_code(err);
}

size_t rtgevc_batched_workspace_size(int32_t count, const int64_t* m, const rtgevc_opts* opts) {
  if (count < 0 || (count > 0 && !m)) return 0;
  for (int i = 0; i < count; ++i)
    if (m[i] < 0) return 0;
  return batch_layout(count, m, opts, nullptr);
}

int rtgevc_batched(int32_t count, const int64_t* m, const double* const* S, const int64_t* lds,
                   const double* const* T, const int64_t* ldt, const int32_t* const* select, double* const* Z,
                   const int64_t* ldz, int32_t* const* scales, int32_t* info, void* work, size_t work_bytes,
                   const rtgevc_opts* opts, void* stream) {
  if (count < 0) return -1;
  if (count == 0) return 0;
  if (!m) return -2;
  if (!S) return -3;
  if (!lds) return -4;
  if (!T) return -5;
  if (!ldt) return -6;
  if (!Z) return -8;
  if (!ldz) return -9;
  if (!opts_ok(opts)) return -14;
  for (int i = 0; i < count; ++i) {
    const int64_t mi = m[i];
    if (mi < 0) return -2;
    if (mi == 0) continue;
    const int64_t lo = mi > 1 ? mi : 1;
    if (!S[i]) return -3;
    if (lds[i] < lo) return -4;
    if (!T[i]) return -5;
    if (ldt[i] < lo) return -6;
    if (!Z[i]) return -8;
    if (ldz[i] < lo) return -9;
  }
  if (!work || (reinterpret_cast<uintptr_t>(work) % kAlign) != 0) return -12;
  std::vector<int64_t> offs(count);
  if (work_bytes < batch_layout(count, m, opts, offs.data())) return -13;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(work);
  PencilDesc* table = reinterpret_cast<PencilDesc*>(base);
  const int normalize = opts ? opts->normalize : 1;
  const int R = batch_band(opts);
  const int split = batch_split(opts);
  std::lock_guard<std::mutex> lock(g_aux_mu);
  Aux* ax = nullptr;
  hipError_t err = get_aux(&ax);
  int first = 0;
  for (int g = 0; g < 3 && err == hipSuccess; ++g) {
    const int mb = kBatchMbs[g];
    // the group's descriptors, in the caller's order
    std::vector<BatchArg> args;
    int64_t max_m = 0;
    int max_tiles = 0;
    for (int i = 0; i < count; ++i) {
      if (m[i] <= 0 || batch_mb(m[i], opts) != mb) continue;
      BatchArg a;
      a.m = m[i];
      a.lds = lds[i];
      a.ldt = ldt[i];
      a.ldz = ldz[i];
      a.off = offs[i];
      a.S = S[i];
      a.T = T[i];
      a.Z = Z[i];
      a.scales = scales ? scales[i] : nullptr;
      a.select = select ? select[i] : nullptr;
      a.info = info ? info + i : nullptr;
      a.mb = mb;
      a.normalize = normalize;
      a.band = R;
      args.push_back(a);
      if (m[i] > max_m) max_m = m[i];
      const int tb = tile_bound(m[i], mb);
      if (tb > max_tiles) max_tiles = tb;
    }
    const int n = (int)args.size();
    if (n == 0) continue;
    for (int c0 = 0; c0 < n; c0 += kSetupPerLaunch) {
      BatchSetup su;
      memset(&su, 0, sizeof(su));
      su.n = (n - c0) < kSetupPerLaunch ? (n - c0) : kSetupPerLaunch;
      su.first = first + c0;
      for (int i = 0; i < su.n; ++i) su.a[i] = args[c0 + i];
      batch_setup_kernel<<<1, kSetupPerLaunch, 0, s>>>(su, table, base);
    }
    const PencilDesc* D = table + first;
    launch_preprocess_batched(D, n, max_m, max_tiles, s);
    // Host bounds of the lock-step: the device's tile count of a pencil is at most
    // tile_bound, so its band of step t starts at most at R (ceil(tile_bound / R) - 1 - t).
    const int steps = (max_tiles + R - 1) / R;
    std::vector<int> above(steps, 0), cr(steps, 0);
    for (int t = 0; t < steps; ++t) {
      int64_t cols = 0;   // tile columns of the step's bands, summed over pencils with rows above
      for (const BatchArg& a : args) {
        const int tb = tile_bound(a.m, mb), b = (tb + R - 1) / R - 1 - t;
        const int nlo = R * b - R;
        if (nlo <= 0) continue;
        above[t] = std::max(above[t], nlo);
        cols += tb - R * b;
      }
      if (split > 0 && cols > 0) cr[t] = (int)std::max<int64_t>(1, (split + cols - 1) / cols);
    }
    struct Ops {
      const PencilDesc* D;
      int n, mb, max_tiles, R;
      hipStream_t st[2];
      hipEvent_t ev[4];
      hipError_t& err;
      bool ok(hipError_t e) {
        if (err == hipSuccess) err = e;
        return err == hipSuccess;
      }
      bool solve(int t, int io, int s) {
        launch_solve_batched(D, n, mb, max_tiles, R, t, io, st[s]);
        return true;
      }
      bool inband(int t, int io, int s) {
        launch_update_batched(D, n, mb, max_tiles, R, t, 0, io, 0, R - 1, st[s]);
        return true;
      }
      bool next(int t, int s) {
        launch_update_batched(D, n, mb, max_tiles, R, t, 1, 0, 0, R, st[s]);
        return true;
      }
      bool above(int t, int off, int cnt, int s) {
        launch_update_batched(D, n, mb, max_tiles, R, t, 2, off, cnt, cnt, st[s]);
        return true;
      }
      bool record(int e, int s) { return ok(hipEventRecord(ev[e], st[s])); }
      bool wait(int s, int e) { return ok(hipStreamWaitEvent(st[s], ev[e], 0)); }
    } ops{D, n, mb, max_tiles, R, {s, ax->side}, {ax->evC, ax->evJ, ax->evU[0], ax->evU[1]}, err};
    batch_band_schedule(steps, R, cr.data(), above.data(), ops);
    launch_consolidate_batched(D, n, max_m, s);
    if (err == hipSuccess) err = hipGetLastError();
    first += n;
  }
  return hip_code(err);
}

int rtgevc_resolve_opts(int64_t m, int32_t batched, const rtgevc_opts* opts, rtgevc_opts* out) {
  if (m < 0) return -1;
  if (!opts_ok(opts)) return -3;
  if (!out) return -4;
  memset(out, 0, sizeof(*out));
  out->normalize = opts ? opts->normalize : 1;
  if (batched) {
    out->mb = batch_mb(m, opts);
    out->band = batch_band(opts);
    out->schedule = 1;
  } else {
    out->mb = resolve_mb(m, opts);
    out->band = resolve_band(m, opts);
    out->schedule = resolve_schedule(m, opts);
  }
  out->precision = opts ? opts->precision : 0;
  const int sweeps = batched ? 0 : resolve_sweeps(opts);
  out->max_refine = sweeps > 0 ? sweeps : -1;
  out->refine_bits = opts ? opts->refine_bits : 0;
  const int split = batched ? batch_split(opts) : resolve_split(m, opts);
  out->split = split > 0 ? split : -1;
  out->grid = opts ? opts->grid : 0;
  return 0;
}

const char* rtgevc_strerror(int code) {
  // -i names argument i of the entry point that returned it
  static const char* const kArg[] = {
      "", "argument 1 (m) is negative or invalid", "argument 2 is NULL or invalid",
      "argument 3 is invalid (a leading dimension below max(1, m)?)", "argument 4 is NULL or invalid",
      "argument 5 is invalid (a leading dimension below max(1, m)?)", "argument 6 is NULL or invalid",
      "argument 7 is NULL or invalid", "argument 8 is NULL or invalid", "argument 9 is NULL or invalid",
      "argument 10 is NULL or invalid", "argument 11 is NULL or invalid (workspace NULL or not 256-byte aligned?)",
      "argument 12 is invalid (workspace too small, or options?)", "argument 13 is invalid (workspace or options?)",
      "argument 14 is invalid (workspace too small?)", "argument 15 is invalid (options or stats?)",
      "argument 16 is invalid"};
  if (code == 0) return "success";
  if (code == RTGEVC_ERR_SCRATCH)
    return "the workspace this order and these options need exceeds the fixed scratch of rtgevc_noalloc "
           "(RTGEVC_NOALLOC_SCRATCH_BYTES); use rtgevc with a workspace";
  if (code <= -1000) return hipGetErrorString(static_cast<hipError_t>(-1000 - code));
  if (code < 0 && code >= -16) return kArg[-code];
  return "invalid argument";
}

const char* rtgevc_version(void) { return "0.1.0"; }

}  // extern "C"
