// Host runtime of libttm: argument validation, workspace planning, the TTM
// schedule of Sec. II.B, and the C ABI declared in include/ttm.h.
//
// Schedule (N sites, 0-based):
//   1. copy the inputs into workspace slots; bring A and B to left-orthonormal
//      form by QR sweeps in their own orientation;
//   2. reverse B (Eq. tensor): B~_i[b, w, a] = B_i[a, w, b]; the chain
//      [A_0 .. A_{N-1}, B~_{N-1} .. B~_0] is then in mixed-canonical gauge;
//   3. contract site N-1 (Eq. contract);
//   4. for j = N-2 .. 0: move the gauge centre from Pi_{j+1} to Pi_{N-1} by
//      QR; move X = B~_j leftwards through Pi_{N-1} .. Pi_{j+1} by Swaps
//      (merge, leg exchange, truncated SVD under Eq. (eps), singular values
//      kept in X so the centre stays inside the next pair); contract A_j
//      with X into Pi_j;
//   5. optionally a left-to-right truncated-SVD sweep with cap chi_out;
//   6. pack the cores into the caller's output buffer.
// Every rank is read back to the host to size the next launches, so the call
// synchronises with its stream once per SVD.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ttm.h"
#include "ttm_internal.h"

namespace ttm {

namespace {
thread_local char g_last_error[512];
}  // namespace

void set_last_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}
void clear_last_error() { g_last_error[0] = '\0'; }
void note_hip_error(hipError_t e, const char *what) {
  set_last_error("%s in %s: %s", hipGetErrorName(e), what ? what : "a HIP call", hipGetErrorString(e));
}
const char *last_error_text() { return g_last_error; }

namespace {

constexpr int64_t kSat = (int64_t)1 << 40;  // saturation of structural products

struct Shape {
  int rl = 1, d = 1, rr = 1;
  int64_t size() const { return (int64_t)rl * d * rr; }
};

struct Options {
  int chi_mid = -1;   // resolved: 0 = uncapped
  int final_round = 1;
  int max_sweeps = 10;
  int svd_max_sweeps = 40;
  uint64_t seed = 12345;
  const int32_t *forced = nullptr;
  int n_forced = 0;
  int trace_cap = 0;
  int32_t *rank_trace = nullptr;
  double *discard_trace = nullptr;
  int profile = 0;
  int contract_prec = GEMM_F64;
  int move_factor = TTM_MOVE_SECOND;
  int gauge = TTM_GAUGE_MOVING;
  int svd_mode = TTM_SVD_JACOBI;
  int rsvd_power = 10;
  double rsvd_tol = 2e-8;
};

// Largest matrix a QR or SVD step takes: each side at most 2^30 (the kernels
// hold dimensions in 32-bit integers and form offsets in 64 bits) and at most
// 2^36 entries, beyond any device memory, so that no size sum can wrap.
constexpr int64_t kMaxSide = (int64_t)1 << 30;
constexpr int64_t kMaxEntries = (int64_t)1 << 36;
bool unfolding_ok(int64_t m, int64_t n) {
  return m >= 1 && n >= 1 && m <= kMaxSide && n <= kMaxSide && m * n <= kMaxEntries;
}

int64_t sat_mul(int64_t a, int64_t b) {
  if (a >= kSat || b >= kSat) return kSat;
  int64_t p = a * b;
  return p > kSat ? kSat : p;
}

// ------------------------------------------------------------------ validation
int validate_tt(const ttm_tt *t) {
  if (!t) return TTM_EINVAL;
  if (t->n_sites < 1 || t->n_sites > 4096) return TTM_EINVAL;
  if (!t->phys || !t->bonds || !t->offsets || !t->data) return TTM_EINVAL;
  if (t->dtype != TTM_F64) return TTM_EUNSUPPORTED;
  if (t->bonds[0] != 1 || t->bonds[t->n_sites] != 1) return TTM_ESHAPE;
  for (int i = 0; i < t->n_sites; ++i) {
    if (t->phys[i] < 1 || t->phys[i] > 65536) return TTM_EINVAL;
    if (t->bonds[i] < 1 || t->bonds[i] > (1 << 20)) return TTM_EINVAL;
    if (t->offsets[i] < 0) return TTM_EINVAL;
  }
  return TTM_OK;
}

int validate_pair(const ttm_tt *A, const ttm_tt *B) {
  int e = validate_tt(A);
  if (e) return e;
  e = validate_tt(B);
  if (e) return e;
  if (A->n_sites != B->n_sites) return TTM_ESHAPE;
  for (int i = 0; i < A->n_sites; ++i)
    if (A->phys[i] != B->phys[i]) return TTM_ESHAPE;
  return TTM_OK;
}

int resolve_options(const ttm_options *o, int chi_out, Options &r) {
  ttm_options d;
  ttm_default_options(&d);
  if (!o) o = &d;
  if (o->chi_mid < -1) return TTM_EINVAL;
  r.chi_mid = (o->chi_mid == -1) ? chi_out : o->chi_mid;
  if (o->final_round != 0 && o->final_round != 1) return TTM_EINVAL;
  r.final_round = o->final_round;
  if (o->max_sweeps < 1 || o->max_sweeps > 10000) return TTM_EINVAL;
  r.max_sweeps = o->max_sweeps;
  if (o->svd_max_sweeps < 1 || o->svd_max_sweeps > 10000) return TTM_EINVAL;
  r.svd_max_sweeps = o->svd_max_sweeps;
  r.seed = o->seed;
  if (o->n_forced < 0) return TTM_EINVAL;
  if (o->n_forced > 0 && !o->forced_ranks) return TTM_EINVAL;
  for (int i = 0; i < o->n_forced; ++i)
    if (o->forced_ranks[i] < 1) return TTM_EFORCED;
  r.forced = o->forced_ranks;
  r.n_forced = o->n_forced;
  if (o->trace_cap < 0) return TTM_EINVAL;
  if (o->trace_cap > 0 && (!o->rank_trace || !o->discard_trace)) return TTM_EINVAL;
  r.trace_cap = o->trace_cap;
  r.rank_trace = o->rank_trace;
  r.discard_trace = o->discard_trace;
  if (o->profile != 0 && o->profile != 1) return TTM_EINVAL;
  r.profile = o->profile;
  if (o->contract_precision < TTM_PREC_F64 || o->contract_precision > TTM_PREC_BF16X3) return TTM_EINVAL;
  r.contract_prec = o->contract_precision;  // TTM_PREC_* and GemmPrec share their values
  if (o->move_factor != TTM_MOVE_SECOND && o->move_factor != TTM_MOVE_SMALLER) return TTM_EINVAL;
  r.move_factor = o->move_factor;
  if (o->svd_mode != TTM_SVD_JACOBI && o->svd_mode != TTM_SVD_RANDOMIZED) return TTM_EINVAL;
  r.svd_mode = o->svd_mode;
  if (o->rsvd_power < 0 || o->rsvd_power > 64) return TTM_EINVAL;
  r.rsvd_power = o->rsvd_power;
  if (!(o->rsvd_tol > 0.0 && o->rsvd_tol <= 1.0)) return TTM_EINVAL;  // also rejects NaN
  r.rsvd_tol = o->rsvd_tol;
  if (o->gauge != TTM_GAUGE_MOVING && o->gauge != TTM_GAUGE_RIGHT) return TTM_EINVAL;
  r.gauge = o->gauge;
  return TTM_OK;
}

// With move_factor = TTM_MOVE_SMALLER the train with the smaller largest
// bond plays the moving (second) factor: returns true when A and B trade
// places.
bool moves_first(const ttm_tt *A, const ttm_tt *B, const Options &o) {
  if (o.move_factor != TTM_MOVE_SMALLER) return false;
  int ma = 1, mb = 1;
  for (int i = 0; i <= A->n_sites; ++i) ma = std::max(ma, A->bonds[i]);
  for (int i = 0; i <= B->n_sites; ++i) mb = std::max(mb, B->bonds[i]);
  return ma < mb;
}

// ------------------------------------------------------------------ planning
// A symbolic run of the schedule with upper bounds in place of ranks.  The
// same caps are applied to the real ranks, so every buffer sized here holds
// whatever the run produces.
struct Plan {
  int n = 0;
  std::vector<int> phys;
  int64_t max_core = 1;  // doubles of the largest core
  int max_bond = 1;
  int64_t max_w = 1;     // doubles of the largest SVD workspace
  int64_t max_qr = 1;    // doubles of the largest QR scratch
  int64_t max_r = 1;     // doubles of the largest R / S V^T factor
  int64_t out_capacity = 0;
  std::vector<Shape> out_shapes;
  size_t ws_bytes = 0;
  int nslots = 0;
  // reverse mode: doubles of the record of every step (upper bound), and
  // the largest SVD matrix (m n doubles)
  int64_t tape = 0;
  int64_t max_mn = 1;
};
int64_t tape_round(int64_t n) { return (n + 31) & ~(int64_t)31; }

// Structural bound of a bond of the product: min(prod_{k<i} d_k, prod_{k>=i} d_k).
int64_t product_bound(const std::vector<int> &phys, int i) {
  int64_t l = 1, r = 1;
  for (int k = 0; k < i; ++k) l = sat_mul(l, phys[k]);
  for (int k = i; k < (int)phys.size(); ++k) r = sat_mul(r, phys[k]);
  return std::min(l, r);
}

// Bound of the bond created by the swap of X (the carriage of site j) with
// Pi_p: its left holds sites 0..j of A, X and Pi_{j+1}..Pi_{p-1}; its right
// holds Pi_p..Pi_{N-1} and B~_{j-1}..B~_0.
int64_t swap_cut_bound(const std::vector<int> &phys, int j, int p) {
  int64_t l = 1, r = 1;
  for (int k = 0; k <= j; ++k) l = sat_mul(l, phys[k]);
  l = sat_mul(l, phys[j]);
  for (int k = j + 1; k < p; ++k) l = sat_mul(l, phys[k]);
  for (int k = p; k < (int)phys.size(); ++k) r = sat_mul(r, phys[k]);
  for (int k = 0; k < j; ++k) r = sat_mul(r, phys[k]);
  return std::min(l, r);
}

int swap_cap(const Options &o, const std::vector<int> &phys, int j, int p, const Shape &P,
             const Shape &X) {
  int64_t c = std::min<int64_t>((int64_t)P.rl * X.d, (int64_t)P.d * X.rr);
  c = std::min(c, swap_cut_bound(phys, j, p));
  if (o.chi_mid > 0) c = std::min<int64_t>(c, o.chi_mid);
  return (int)c;
}

int round_cap(int chi_out, const std::vector<int> &phys, int i, const Shape &M) {
  int64_t c = std::min<int64_t>((int64_t)M.rl * M.d, M.rr);
  c = std::min(c, product_bound(phys, i + 1));
  c = std::min<int64_t>(c, chi_out);
  return (int)c;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

void note_core(Plan &pl, const Shape &s) {
  pl.max_core = std::max(pl.max_core, s.size());
  pl.max_bond = std::max(pl.max_bond, std::max(s.rl, s.rr));
}
// Workspace of one truncated SVD of an np x no matrix; `own_y` adds room for
// the matrix itself (the swap builds it there).  False when np (the side
// whose singular vectors come out orthonormal, which also bounds the Jacobi
// size) exceeds what the SVD kernels take.
bool note_svd(Plan &pl, int np, int no, bool own_y) {
  if (np > kSvdMaxSide) return false;
  SvdPlan sp = svd_plan(np, no);
  int64_t need = (int64_t)svd_ws_doubles(sp);
  if (own_y) need += (((int64_t)np * no + 31) & ~(int64_t)31);
  pl.max_w = std::max<int64_t>(pl.max_w, need);
  return true;
}
void note_qr(Plan &pl, int m, int n) {
  pl.max_qr = std::max<int64_t>(pl.max_qr, (int64_t)qr_scratch_doubles(m, n));
  const int k = std::min(m, n);
  pl.max_r = std::max<int64_t>(pl.max_r, (int64_t)k * n);
}

int make_plan(const ttm_tt *A, const ttm_tt *B, int chi_out, const Options &o, Plan &pl) {
  if (moves_first(A, B, o)) std::swap(A, B);
  const int n = A->n_sites;
  pl.n = n;
  pl.phys.assign(A->phys, A->phys + n);
  std::vector<Shape> a(n), b(n), pi(n);
  for (int i = 0; i < n; ++i) {
    a[i] = {A->bonds[i], A->phys[i], A->bonds[i + 1]};
    b[i] = {B->bonds[i], B->phys[i], B->bonds[i + 1]};
    note_core(pl, a[i]);
    note_core(pl, b[i]);
  }
  auto tape_qr = [&](int64_t m, int64_t nn, int64_t ncol) {
    const int64_t k = std::min(m, nn);
    pl.tape += tape_round(m * nn) + tape_round(m * k) + tape_round(k * nn) + tape_round(nn * ncol);
  };
  auto qr_sweep = [&](std::vector<Shape> &t) {
    for (int i = 0; i + 1 < n; ++i) {
      if (!unfolding_ok((int64_t)t[i].rl * t[i].d, t[i].rr)) return false;
      const int m = t[i].rl * t[i].d, nn = t[i].rr;
      note_qr(pl, m, nn);
      tape_qr(m, nn, (int64_t)t[i + 1].d * t[i + 1].rr);
      const int k = std::min(m, nn);
      t[i].rr = k;
      t[i + 1].rl = k;
      note_core(pl, t[i]);
      note_core(pl, t[i + 1]);
    }
    return true;
  };
  if (!qr_sweep(a) || !qr_sweep(b)) return TTM_EINVAL;
  std::vector<Shape> bt(n);
  for (int i = 0; i < n; ++i) bt[i] = {b[i].rr, b[i].d, b[i].rl};
  pi[n - 1] = {a[n - 1].rl, a[n - 1].d, bt[n - 1].rr};
  note_core(pl, pi[n - 1]);
  pl.tape += tape_round(a[n - 1].size()) + tape_round(bt[n - 1].size());
  for (int j = n - 2; j >= 0; --j) {
    for (int p = j + 1; p <= n - 2; ++p) {
      if (!unfolding_ok((int64_t)pi[p].rl * pi[p].d, pi[p].rr)) return TTM_EINVAL;
      const int m = pi[p].rl * pi[p].d, nn = pi[p].rr;
      note_qr(pl, m, nn);
      tape_qr(m, nn, (int64_t)pi[p + 1].d * pi[p + 1].rr);
      const int k = std::min(m, nn);
      pi[p].rr = k;
      pi[p + 1].rl = k;
      note_core(pl, pi[p]);
      note_core(pl, pi[p + 1]);
    }
    Shape x = bt[j];
    for (int p = n - 1; p > j; --p) {
      if (!unfolding_ok((int64_t)pi[p].rl * x.d, (int64_t)pi[p].d * x.rr)) return TTM_EINVAL;
      const int m = pi[p].rl * x.d, nn = pi[p].d * x.rr;
      const int r = swap_cap(o, pl.phys, j, p, pi[p], x);
      if (o.gauge == TTM_GAUGE_RIGHT) {
        // SVD with the orthonormal factor over the rows (a, w), then the LQ of
        // S_r V_r^T (r x nn): a QR of its transpose and the r x r factor
        if (!note_svd(pl, nn, m, true)) return TTM_EUNSUPPORTED;
        note_qr(pl, nn, r);
      } else if (!note_svd(pl, m, nn, true)) {
        return TTM_EUNSUPPORTED;
      }
      if (o.gauge != TTM_GAUGE_RIGHT && o.svd_mode == TTM_SVD_RANDOMIZED && !o.forced && rsvd_eligible(m, nn, r))
        pl.max_w = std::max<int64_t>(pl.max_w, (int64_t)rsvd_ws_doubles(m, nn, r) +
                                                   ((((int64_t)m * nn) + 31) & ~(int64_t)31));
      Shape xn = {pi[p].rl, x.d, r};
      Shape pn = {r, pi[p].d, x.rr};
      note_core(pl, xn);
      note_core(pl, pn);
      {
        const int64_t mm = m, nnn = nn, kk = std::min(mm, nnn);
        pl.max_mn = std::max(pl.max_mn, mm * nnn);
        pl.tape += tape_round(pi[p].size()) + tape_round(x.size()) + tape_round(mm * nnn) +
                   tape_round(nnn * kk) + tape_round(kk) + tape_round(mm * r);
      }
      x = xn;
      pi[p] = pn;
    }
    pi[j] = {a[j].rl, a[j].d, x.rr};
    note_core(pl, pi[j]);
    pl.tape += tape_round(a[j].size()) + tape_round(x.size());
  }
  if (o.final_round) {
    for (int i = 0; i + 1 < n; ++i) {
      if (!unfolding_ok((int64_t)pi[i].rl * pi[i].d, pi[i].rr)) return TTM_EINVAL;
      const int m = pi[i].rl * pi[i].d, nn = pi[i].rr;
      if (!note_svd(pl, nn, m, false)) return TTM_EUNSUPPORTED;
      const int r = round_cap(chi_out, pl.phys, i, pi[i]);
      pl.max_r = std::max<int64_t>(pl.max_r, (int64_t)r * nn);
      {
        const int64_t mm = m, nnn = nn, kk = std::min(mm, nnn);
        pl.max_mn = std::max(pl.max_mn, mm * nnn);
        pl.tape += tape_round(mm * nnn) + tape_round(mm * kk) + tape_round(kk) + tape_round((int64_t)r * nnn) +
                   tape_round(nnn * (int64_t)pi[i + 1].d * pi[i + 1].rr);
      }
      pi[i].rr = r;
      pi[i + 1].rl = r;
      note_core(pl, pi[i]);
      note_core(pl, pi[i + 1]);
    }
  }
  pl.out_shapes = pi;
  pl.out_capacity = 0;
  for (int i = 0; i < n; ++i) pl.out_capacity += pi[i].size();
  // Slots: A (N) + B (N) + B~/Pi (N) + X + 3 spares (4 when each swap also
  // runs an LQ move: its Q and the moved carriage are held at once).
  pl.nslots = 3 * n + (o.gauge == TTM_GAUGE_RIGHT ? 5 : 4);
  size_t bytes = 0;
  bytes += (size_t)pl.nslots * align_up((size_t)pl.max_core * 8);
  bytes += align_up((size_t)pl.max_w * 8);
  bytes += align_up((size_t)pl.max_qr * 8);
  bytes += align_up((size_t)pl.max_r * 8);
  bytes += 256;  // flags
  pl.ws_bytes = bytes;
  if (pl.max_bond > (1 << 20) || pl.max_core > ((int64_t)1 << 33)) return TTM_EINVAL;
  return TTM_OK;
}

// ------------------------------------------------------------------ device state
struct Core {
  double *p = nullptr;
  Shape s;
};

struct Runner {
  hipStream_t st;
  const Options &o;
  std::vector<double *> free_slots;
  double *wbuf = nullptr, *qrbuf = nullptr, *rbuf = nullptr;
  int *flags = nullptr;
  int64_t max_core = 0;
  int trace = 0;  // TTM_TRACE: 1 = one line per step, 2 = also one per Jacobi sweep
  // stats
  int n_contract = 0, n_swap = 0, n_qr = 0, n_svd = 0, n_trace = 0, max_bond = 1;
  int64_t n_rsvd = 0;  // randomized SVDs started (each takes its own stretch of the random stream)
  int n_rsvd_done = 0, n_rsvd_fallback = 0;
  int jac_sweeps = 0, jac_max = 0;
  double disc_sum = 0.0, err_bound = 0.0, flops = 0.0, svd_flops = 0.0, solve_flops = 0.0;
  int forced_pos = 0;
  int err = TTM_OK;
  KernelTimer timer;
  Tape *tape = nullptr;  // reverse mode: record every step's operands

  void tape_full() {
    if (err == TTM_OK) {
      err = TTM_EWORKSPACE;
      set_last_error("the reverse-mode record outgrew its workspace region");
    }
  }
  // A device copy of n doubles in the tape region.
  double *keep(const double *src, int64_t n) {
    double *dst = tape->alloc((size_t)n);
    if (!dst) {
      tape_full();
      return nullptr;
    }
    hip(launch_copy(dst, src, n, st));
    return dst;
  }

  Runner(hipStream_t s, const Options &opt) : st(s), o(opt) {
    const char *tv = getenv("TTM_TRACE");
    trace = tv ? (atoi(tv) > 0 ? atoi(tv) : 1) : 0;
    timer.on = opt.profile != 0;
  }
  // synchronise the stream and read the event timers
  bool sync() {
    if (!hip(hipStreamSynchronize(st))) return false;
    if (timer.on) timer.collect();
    return true;
  }

  double *take() {
    if (free_slots.empty()) {
      err = TTM_EINVAL;  // planning error: never expected
      return nullptr;
    }
    double *p = free_slots.back();
    free_slots.pop_back();
    return p;
  }
  void give(double *p) {
    if (p) free_slots.push_back(p);
  }
  bool hip(hipError_t e) {
    if (e != hipSuccess) {
      if (err == TTM_OK) {
        err = TTM_EHIP;
        note_hip_error(e, step);
      }
      if (trace) fprintf(stderr, "[ttm] HIP error %s (%s) in %s\n", hipGetErrorName(e), hipGetErrorString(e), step);
      return false;
    }
    return true;
  }
  // the step being enqueued, for error messages
  const char *step = "the set-up of a TTM product";
  void note(const Shape &s) { max_bond = std::max(max_bond, std::max(s.rl, s.rr)); }

  // ---- Eq. (contract): out[a, e, b] = sum_c K[a, e, c] M[c, e, b]
  Core contract(const Core &k, const Core &m, int site = 0) {
    step = "a contraction (Eq. contract)";
    if (tape) {
      TapeEntry e;
      e.kind = TapeEntry::CONTRACT;
      e.p = site;
      e.dl = k.s.rl; e.d = k.s.d; e.dm = k.s.rr; e.dr = m.s.rr;
      e.K = keep(k.p, k.s.size());
      e.X = keep(m.p, m.s.size());
      tape->e.push_back(e);
    }
    Core out;
    out.p = take();
    out.s = {k.s.rl, k.s.d, m.s.rr};
    if (!out.p) return out;
    GemmArgs g;
    g.M = k.s.rl; g.N = m.s.rr; g.K = k.s.rr; g.batch = k.s.d;
    g.A = k.p; g.a_rs = (int64_t)k.s.d * k.s.rr; g.a_cs = 1; g.a_bs = k.s.rr;
    g.B = m.p; g.b_rs = (int64_t)m.s.d * m.s.rr; g.b_cs = 1; g.b_bs = m.s.rr;
    g.C = out.p; g.c_rs1 = (int64_t)k.s.d * m.s.rr; g.c_cs1 = 1; g.c_bs = m.s.rr;
    g.prec = o.contract_prec;
    {
      Timed tm(&timer, KC_GEMM, st);
      hip(launch_gemm(g, st));
    }
    flops += 2.0 * k.s.d * k.s.rl * k.s.rr * m.s.rr;
    ++n_contract;
    note(out.s);
    if (trace) fprintf(stderr, "[ttm] contract %dx%dx%d * %dx%dx%d\n", k.s.rl, k.s.d, k.s.rr, m.s.rl, m.s.d, m.s.rr);
    return out;
  }

  // ---- gauge move: QR of cores[p], R into cores[p+1]
  void qr_move(std::vector<Core> &c, int p, int arr = 2) {
    step = "a QR gauge move";
    Core &cur = c[p];
    Core &nxt = c[p + 1];
    const int m = cur.s.rl * cur.s.d, n = cur.s.rr;
    const int k = std::min(m, n);
    TapeEntry e;
    if (tape) {
      e.kind = TapeEntry::QR;
      e.arr = arr;
      e.p = p;
      e.m = m; e.n = n; e.k = k; e.ncol = nxt.s.d * nxt.s.rr;
      e.rl = cur.s.rl; e.d = cur.s.d;
      e.M = keep(cur.p, (int64_t)m * n);
      e.nxt = keep(nxt.p, (int64_t)n * e.ncol);
    }
    double *q = take();
    if (!q) return;
    {
      Timed tm(&timer, KC_QR, st);
      hip(launch_qr(cur.p, m, n, n, 1, q, rbuf, qrbuf, st));
    }
    if (tape) {
      e.Q = keep(q, (int64_t)m * k);
      e.R = keep(rbuf, (int64_t)k * n);
      tape->e.push_back(e);
    }
    double *nn = take();
    if (!nn) return;
    const int ncol = nxt.s.d * nxt.s.rr;
    {
      Timed tm(&timer, KC_GEMM, st);
      hip(launch_gemm(gemm_rowmajor(k, ncol, n, rbuf, n, nxt.p, ncol, nn, ncol), st));
    }
    give(cur.p);
    give(nxt.p);
    cur.p = q;
    cur.s.rr = k;
    nxt.p = nn;
    nxt.s.rl = k;
    ++n_qr;
    flops += (m >= n) ? 4.0 * m * n * (double)n - (4.0 / 3.0) * n * (double)n * n
                      : 2.0 * n * m * (double)m + (2.0 / 3.0) * m * (double)m * m;
    flops += 2.0 * k * n * (double)ncol;
    note(cur.s);
    note(nxt.s);
  }

  // ---- one truncated SVD (svd_oside) with the bookkeeping of the rule of
  // Eq. (eps): forced ranks, traces, discarded weight and the flop model.
  // Returns the rank, or -1 after setting err.
  int svd(const SvdPlan &sp, const double *Y, double *ws, int cap, double *u, int u_layout, SvdAll *all = nullptr) {
    int forced = 0;
    if (o.forced) {
      if (forced_pos >= o.n_forced) {
        err = TTM_EFORCED;
        return -1;
      }
      forced = o.forced[forced_pos++];
      // a forced rank may not exceed what the buffers were sized for
      if (forced > std::min(sp.k, cap)) {
        err = TTM_EFORCED;
        return -1;
      }
    }
    SvdResult so = svd_oside(sp, Y, eps_, cap, forced, o.svd_max_sweeps, u, u_layout, nullptr, ws, st, &timer,
                             trace, all);
    jac_sweeps += so.sweeps;
    jac_max = std::max(jac_max, so.sweeps);
    if (so.err != TTM_OK) {
      if (err == TTM_OK) err = so.err;
      return -1;
    }
    ++n_svd;
    disc_sum += so.disc;
    err_bound += sqrt(std::max(so.disc, 0.0));
    if (n_trace < o.trace_cap) {
      o.rank_trace[n_trace] = so.rank;
      o.discard_trace[n_trace] = so.disc;
    }
    ++n_trace;
    const int m = std::max(sp.np, sp.no), n = std::min(sp.np, sp.no);
    const double f = 4.0 * m * (double)n * n - (4.0 / 3.0) * n * (double)n * n + 4.0 * (m + n) * (double)n * so.rank;
    flops += f;
    svd_flops += f;
    // the solve kernel's own arithmetic per pair and launch: the sum of gsw
    // partial Grams, B2 - 1 rotation steps (6 flops per entry of G and Q),
    // and two B2^3 products of the re-orthogonalisation
    {
      const JacobiPlan &jp = sp.jp;
      const double b2 = 2.0 * jp.bw;
      const double per_pair = jp.gsw * b2 * b2 + 6.0 * b2 * b2 * (b2 - 1.0) + 4.0 * b2 * b2 * b2;
      solve_flops += (double)so.sweeps * jp.rounds * jp.pairs * per_pair;
    }
    return so.rank;
  }

  // ---- the randomized truncated SVD of a swap matrix (svd_mode
  // TTM_SVD_RANDOMIZED) with the same bookkeeping as svd(); *done = false
  // when it fell back (CholeskyQR breakdown) and the full SVD must run.
  int rsvd(const double *Y, int m, int n, int cap, double *pt, double *ws, bool *done) {
    *done = false;
    RsvdResult rs = rsvd_oside(Y, m, n, cap, o.rsvd_power, o.rsvd_tol, o.svd_max_sweeps, eps_, o.contract_prec,
                               o.seed, (int64_t)n_rsvd << 40, pt, ws, st, &timer, trace);
    ++n_rsvd;
    jac_sweeps += rs.sweeps;
    jac_max = std::max(jac_max, rs.sweeps);
    if (rs.err != TTM_OK) {
      if (err == TTM_OK) err = rs.err;
      return -1;
    }
    if (rs.fallback) {
      ++n_rsvd_fallback;
      return 0;
    }
    *done = true;
    ++n_rsvd_done;
    ++n_svd;
    disc_sum += rs.disc;
    err_bound += sqrt(std::max(rs.disc, 0.0));
    if (n_trace < o.trace_cap) {
      o.rank_trace[n_trace] = rs.rank;
      o.discard_trace[n_trace] = rs.disc;
    }
    ++n_trace;
    flops += rs.flops;
    svd_flops += rs.flops;
    return rs.rank;
  }

  // ---- Swap of Fig. 1C: (P, X) -> (X', P') with X' = U_r S_r, P' = V_r^T.
  void swap(Core &P, Core &X, int cap, int pos = 0, int site = 0) {
    step = "a swap";
    if (o.gauge == TTM_GAUGE_RIGHT) {
      swap_centre_right(P, X, cap);
      return;
    }
    const int Dl = P.s.rl, dp = P.s.d, Dm = P.s.rr, dx = X.s.d, Dr = X.s.rr;
    const int m = Dl * dx, n = dp * Dr;
    const SvdPlan sp = svd_plan(m, n);
    TapeEntry e;
    SvdAll all;
    if (tape) {
      e.kind = TapeEntry::SWAP;
      e.p = pos;
      e.j = site;
      e.dl = Dl; e.dp = dp; e.dm = Dm; e.dx = dx; e.dr = Dr;
      e.m = m; e.n = n; e.k = sp.k;
      e.P = keep(P.p, P.s.size());
      e.X = keep(X.p, X.s.size());
      e.V = tape->alloc((size_t)n * sp.k);
      e.sigma = tape->alloc((size_t)sp.k);
      if (!e.V || !e.sigma) {
        tape_full();
        return;
      }
      all.u = e.V;
      all.sigma = e.sigma;
    }
    double *Y = wbuf;
    double *sws = wbuf + ((((int64_t)m * n) + 31) & ~(int64_t)31);
    // merge: theta[(a,e),(w,b)] = sum_c P[a,e,c] X[c,w,b], stored as the
    // leg-exchanged unfolding Theta[(a,w),(e,b)], column-major (ld m).
    GemmArgs g;
    g.M = Dl * dp; g.N = dx * Dr; g.K = Dm;
    g.A = P.p; g.a_rs = Dm; g.a_cs = 1;
    g.B = X.p; g.b_rs = (int64_t)dx * Dr; g.b_cs = 1;
    g.C = Y;
    g.c_rdiv = dp; g.c_cdiv = Dr;
    g.c_rs1 = dx; g.c_rs0 = (int64_t)m * Dr; g.c_cs1 = 1; g.c_cs0 = m;
    g.prec = o.contract_prec;
    {
      Timed tm(&timer, KC_GEMM, st);
      if (!hip(launch_gemm(g, st))) return;
    }
    flops += 2.0 * Dl * dp * (double)Dm * dx * Dr;
    double *xn = take();
    double *pn = take();
    if (!xn || !pn) return;
    if (tape) e.theta = keep(Y, (int64_t)m * n);
    // P' = V_r^T -> [r, dp, Dr] (the orthonormal factor, over Theta's columns)
    int r = 0;
    bool done = false;
    if (o.svd_mode == TTM_SVD_RANDOMIZED && !o.forced && !tape && rsvd_eligible(m, n, cap)) {
      r = rsvd(Y, m, n, cap, pn, sws, &done);
      if (r < 0) return;
    }
    if (!done) r = svd(sp, Y, sws, cap, pn, SVD_U_T, tape ? &all : nullptr);
    if (r < 1) return;
    // X' = Theta V_r = U_r S_r -> [Dl, dx, r]
    GemmArgs z;
    z.M = m; z.N = r; z.K = n;
    z.A = Y; z.a_rs = 1; z.a_cs = m;
    z.B = pn; z.b_rs = 1; z.b_cs = n;
    z.C = xn; z.c_rs1 = r; z.c_cs1 = 1;
    {
      Timed tm(&timer, KC_GEMM, st);
      if (!hip(launch_gemm(z, st))) return;
    }
    if (tape) {
      e.r = r;
      e.kg = all.kg;
      e.Z = keep(xn, (int64_t)m * r);
      tape->e.push_back(e);
    }
    give(P.p);
    give(X.p);
    X.p = xn;
    X.s = {Dl, dx, r};
    P.p = pn;
    P.s = {r, dp, Dr};
    ++n_swap;
    note(X.s);
    note(P.s);
  }

  // ---- The swap with the centre put where Sec. II.B puts it: the singular
  // values go to the right carriage, X' = U_r and P' = S_r V_r^T; then an LQ
  // factorisation P' = L Q moves the centre into the carriage that moves on
  // (X' <- X' L, P' <- Q), so that the next pair holds it.  In exact
  // arithmetic L Q = S_r V_r^T with L = S_r (up to signs), and the result is
  // the one of the default gauge.
  void swap_centre_right(Core &P, Core &X, int cap) {
    const int Dl = P.s.rl, dp = P.s.d, Dm = P.s.rr, dx = X.s.d, Dr = X.s.rr;
    const int m = Dl * dx, n = dp * Dr;
    // Theta row-major (m x n) is the column-major n x m matrix Theta^T, whose
    // right singular vectors are Theta's left ones.
    const SvdPlan sp = svd_plan(n, m);
    double *Y = wbuf;
    double *sws = wbuf + ((((int64_t)m * n) + 31) & ~(int64_t)31);
    GemmArgs g;
    g.M = Dl * dp; g.N = dx * Dr; g.K = Dm;
    g.A = P.p; g.a_rs = Dm; g.a_cs = 1;
    g.B = X.p; g.b_rs = (int64_t)dx * Dr; g.b_cs = 1;
    g.C = Y;
    g.c_rdiv = dp; g.c_cdiv = Dr;
    g.c_rs1 = (int64_t)dx * n; g.c_rs0 = Dr; g.c_cs1 = n; g.c_cs0 = 1;
    g.prec = o.contract_prec;
    {
      Timed tm(&timer, KC_GEMM, st);
      if (!hip(launch_gemm(g, st))) return;
    }
    flops += 2.0 * Dl * dp * (double)Dm * dx * Dr;
    double *xn = take();
    double *pn = take();
    if (!xn || !pn) return;
    // X' = U_r -> [Dl, dx, r] (orthonormal over the rows (a, w))
    const int r = svd(sp, Y, sws, cap, xn, SVD_U);
    if (r < 1) return;
    // P' = U_r^T Theta = S_r V_r^T -> [r, dp, Dr]
    GemmArgs z;
    z.M = r; z.N = n; z.K = m;
    z.A = xn; z.a_rs = 1; z.a_cs = r;
    z.B = Y; z.b_rs = n; z.b_cs = 1;
    z.C = pn; z.c_rs1 = n; z.c_cs1 = 1;
    {
      Timed tm(&timer, KC_GEMM, st);
      if (!hip(launch_gemm(z, st))) return;
    }
    // LQ of P' through the QR of its transpose: P'^T = Q R, so P' = R^T Q^T
    double *q = take();
    double *xl = take();
    if (!q || !xl) return;
    {
      Timed tm(&timer, KC_QR, st);
      if (!hip(launch_qr(pn, n, r, 1, n, q, rbuf, qrbuf, st))) return;
    }
    {
      Timed tm(&timer, KC_OTHER, st);
      if (!hip(launch_transpose(pn, q, n, r, st))) return;  // P' <- Q^T (r x n)
    }
    GemmArgs h;  // X' <- X' R^T (m x r)
    h.M = m; h.N = r; h.K = r;
    h.A = xn; h.a_rs = r; h.a_cs = 1;
    h.B = rbuf; h.b_rs = 1; h.b_cs = r;
    h.C = xl; h.c_rs1 = r; h.c_cs1 = 1;
    {
      Timed tm(&timer, KC_GEMM, st);
      if (!hip(launch_gemm(h, st))) return;
    }
    ++n_qr;
    flops += 4.0 * n * (double)r * r - (4.0 / 3.0) * r * (double)r * r;
    flops += 2.0 * m * (double)r * r;
    give(q);
    give(xn);
    give(P.p);
    give(X.p);
    X.p = xl;
    X.s = {Dl, dx, r};
    P.p = pn;
    P.s = {r, dp, Dr};
    ++n_swap;
    note(X.s);
    note(P.s);
  }

  // ---- final rounding step at site i: Pi_i <- U_r, Pi_{i+1} <- S_r V_r^T Pi_{i+1}
  void round_step(std::vector<Core> &c, int i, int cap) {
    step = "a step of the final rounding sweep";
    Core &cur = c[i];
    Core &nxt = c[i + 1];
    const int m = cur.s.rl * cur.s.d, n = cur.s.rr;
    // The row-major m x n core is the column-major n x m matrix Y = Pi_i^T,
    // whose right singular vectors are Pi_i's left ones.
    const SvdPlan sp = svd_plan(n, m);
    TapeEntry e;
    SvdAll all;
    if (tape) {
      e.kind = TapeEntry::ROUND;
      e.p = i;
      e.m = m; e.n = n; e.k = sp.k; e.ncol = nxt.s.d * nxt.s.rr;
      e.rl = cur.s.rl; e.d = cur.s.d;
      e.M = keep(cur.p, (int64_t)m * n);
      e.nxt = keep(nxt.p, (int64_t)n * e.ncol);
      e.V = tape->alloc((size_t)m * sp.k);
      e.sigma = tape->alloc((size_t)sp.k);
      if (!e.V || !e.sigma) {
        tape_full();
        return;
      }
      all.u = e.V;
      all.sigma = e.sigma;
    }
    double *un = take();
    double *nn = take();
    if (!un || !nn) return;
    const int r = svd(sp, cur.p, wbuf, cap, un, SVD_U, tape ? &all : nullptr);
    if (r < 1) return;
    // S_r V_r^T = U_r^T Pi_i  (r x n), then into the next core
    GemmArgs h;
    h.M = r; h.N = n; h.K = m;
    h.A = un; h.a_rs = 1; h.a_cs = r;
    h.B = cur.p; h.b_rs = n; h.b_cs = 1;
    h.C = rbuf; h.c_rs1 = n; h.c_cs1 = 1;
    const int ncol = nxt.s.d * nxt.s.rr;
    {
      Timed tm(&timer, KC_GEMM, st);
      if (!hip(launch_gemm(h, st))) return;
      if (!hip(launch_gemm(gemm_rowmajor(r, ncol, n, rbuf, n, nxt.p, ncol, nn, ncol), st))) return;
    }
    if (tape) {
      e.r = r;
      e.kg = all.kg;
      e.Zt = keep(rbuf, (int64_t)r * n);
      tape->e.push_back(e);
    }
    flops += 2.0 * r * (double)n * ncol;
    give(cur.p);
    give(nxt.p);
    cur.p = un;
    cur.s.rr = r;
    nxt.p = nn;
    nxt.s.rl = r;
    note(cur.s);
    note(nxt.s);
  }

  double eps_ = 0.0;
};

int run_ttm_impl(const ttm_tt *A, const ttm_tt *B, int chi_out, double tol, ttm_tt_out *C, void *ws,
                 size_t ws_bytes, hipStream_t st, const Options &o, ttm_stats *stats, bool &enqueued,
                 Tape *tape = nullptr) {
  Plan pl;
  int e = make_plan(A, B, chi_out, o, pl);
  if (e) return e;
  if (!ws || ws_bytes < pl.ws_bytes) return TTM_EWORKSPACE;
  // the factor that moves plays B (make_plan made the same choice)
  if (moves_first(A, B, o)) std::swap(A, B);
  if (!C || !C->bonds || !C->offsets || !C->data) return TTM_EINVAL;
  if (C->capacity < pl.out_capacity) return TTM_ECAPACITY;
  const int n = pl.n;

  Runner R(st, o);
  R.eps_ = tol;
  R.tape = tape;
  enqueued = true;
  char *base = static_cast<char *>(ws);
  size_t off = 0;
  const size_t slot_bytes = align_up((size_t)pl.max_core * 8);
  for (int i = 0; i < pl.nslots; ++i) {
    R.free_slots.push_back(reinterpret_cast<double *>(base + off));
    off += slot_bytes;
  }
  std::reverse(R.free_slots.begin(), R.free_slots.end());
  R.wbuf = reinterpret_cast<double *>(base + off);
  off += align_up((size_t)pl.max_w * 8);
  R.qrbuf = reinterpret_cast<double *>(base + off);
  off += align_up((size_t)pl.max_qr * 8);
  R.rbuf = reinterpret_cast<double *>(base + off);
  off += align_up((size_t)pl.max_r * 8);
  R.flags = reinterpret_cast<int *>(base + off);
  off += 256;

  const double *Ad = static_cast<const double *>(A->data);
  const double *Bd = static_cast<const double *>(B->data);
  std::vector<Core> a(n), b(n), pi(n);
  R.hip(launch_zero_int(R.flags, 4, st));
  for (int i = 0; i < n; ++i) {
    a[i].s = {A->bonds[i], A->phys[i], A->bonds[i + 1]};
    b[i].s = {B->bonds[i], B->phys[i], B->bonds[i + 1]};
    a[i].p = R.take();
    b[i].p = R.take();
    if (R.err) return R.err;
    Timed tm(&R.timer, KC_OTHER, st);
    R.hip(launch_copy(a[i].p, Ad + A->offsets[i], a[i].s.size(), st));
    R.hip(launch_copy(b[i].p, Bd + B->offsets[i], b[i].s.size(), st));
    R.hip(launch_nonfinite_check(a[i].p, a[i].s.size(), R.flags, st));
    R.hip(launch_nonfinite_check(b[i].p, b[i].s.size(), R.flags, st));
    R.note(a[i].s);
    R.note(b[i].s);
  }
  {
    int hflag[4] = {0, 0, 0, 0};
    R.hip(hipMemcpyAsync(hflag, R.flags, sizeof(hflag), hipMemcpyDeviceToHost, st));
    R.sync();
    if (R.err) return R.err;
    if (hflag[0]) return TTM_ENONFINITE;
  }
  // 1. canonical form of both inputs
  for (int i = 0; i + 1 < n && !R.err; ++i) R.qr_move(a, i, 0);
  for (int i = 0; i + 1 < n && !R.err; ++i) R.qr_move(b, i, 1);
  // 2. reversal of B
  std::vector<Core> bt(n);
  for (int i = 0; i < n && !R.err; ++i) {
    bt[i].p = R.take();
    bt[i].s = {b[i].s.rr, b[i].s.d, b[i].s.rl};
    if (!bt[i].p) break;
    Timed tm(&R.timer, KC_OTHER, st);
    R.hip(launch_reverse_core(bt[i].p, b[i].p, b[i].s.rl, b[i].s.d, b[i].s.rr, st));
    R.give(b[i].p);
    b[i].p = nullptr;
  }
  if (R.err) return R.err;
  if (tape) {
    TapeEntry e;
    e.kind = TapeEntry::REVERSE;
    tape->e.push_back(e);
  }
  // 3. contract site N-1
  pi[n - 1] = R.contract(a[n - 1], bt[n - 1], n - 1);
  R.give(a[n - 1].p);
  R.give(bt[n - 1].p);
  // 4. swaps and contractions
  for (int j = n - 2; j >= 0 && !R.err; --j) {
    for (int p = j + 1; p <= n - 2 && !R.err; ++p) R.qr_move(pi, p);
    Core x = bt[j];
    for (int p = n - 1; p > j && !R.err; --p) {
      const int cap = swap_cap(o, pl.phys, j, p, pi[p].s, x.s);
      R.swap(pi[p], x, cap, p, j);
    }
    if (R.err) break;
    pi[j] = R.contract(a[j], x, j);
    R.give(a[j].p);
    R.give(x.p);
  }
  // 5. final rounding sweep
  if (o.final_round) {
    for (int i = 0; i + 1 < n && !R.err; ++i) {
      const int cap = round_cap(chi_out, pl.phys, i, pi[i].s);
      R.round_step(pi, i, cap);
    }
  }
  if (R.err) return R.err;
  if (o.forced && R.forced_pos != o.n_forced) {
    // extra forced ranks are an inconsistency of the caller's schedule
    return TTM_EFORCED;
  }
  // 6. pack
  int64_t pos = 0;
  for (int i = 0; i < n; ++i) pos += pi[i].s.size();
  if (pos > C->capacity) return TTM_ECAPACITY;
  pos = 0;
  double *Cd = static_cast<double *>(C->data);
  for (int i = 0; i < n; ++i) {
    C->offsets[i] = pos;
    C->bonds[i] = pi[i].s.rl;
    Timed tm(&R.timer, KC_OTHER, st);
    R.hip(launch_copy(Cd + pos, pi[i].p, pi[i].s.size(), st));
    pos += pi[i].s.size();
  }
  C->bonds[n] = pi[n - 1].s.rr;
  R.sync();
  if (R.err) return R.err;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->max_bond = R.max_bond;
    stats->n_contract = R.n_contract;
    stats->n_swap = R.n_swap;
    stats->n_qr = R.n_qr;
    stats->n_svd = R.n_svd;
    stats->n_trace = std::min(R.n_trace, o.trace_cap);
    stats->sweeps = R.jac_sweeps;
    stats->jacobi_max_sweeps = R.jac_max;
    stats->discarded_sq_sum = R.disc_sum;
    stats->error_bound = R.err_bound;
    stats->model_flops = R.flops;
    stats->svd_model_flops = R.svd_flops;
    stats->jacobi_solve_flops = R.solve_flops;
    stats->peak_ws_bytes = pl.ws_bytes;
    stats->n_rsvd = R.n_rsvd_done;
    stats->n_rsvd_fallback = R.n_rsvd_fallback;
    for (int c = 0; c < KC_COUNT; ++c) {
      stats->kernel_ms[c] = R.timer.ms[c];
      stats->kernel_launches[c] = R.timer.launches[c];
    }
  }
  return TTM_OK;
}

}  // namespace

// The product with its reverse-mode record (used by ttm_multiply_vjp): the
// schedule of run_ttm with every step's operands copied into `tape`.
int run_ttm_taped(const ttm_tt *A, const ttm_tt *B, int chi_out, double tol, const ttm_options *opt,
                  ttm_tt_out *C, void *ws, size_t ws_bytes, hipStream_t st, ttm_stats *stats, Tape *tape,
                  bool *swapped) {
  Options o;
  int e = resolve_options(opt, chi_out, o);
  if (e) return e;
  // the reverse mode differentiates the full SVD's truncation only
  if (o.gauge != TTM_GAUGE_MOVING || o.svd_mode != TTM_SVD_JACOBI) return TTM_EUNSUPPORTED;
  *swapped = moves_first(A, B, o);
  bool enqueued = false;
  e = run_ttm_impl(A, B, chi_out, tol, C, ws, ws_bytes, st, o, stats, enqueued, tape);
  if (e == TTM_OK && tape->overflow) e = TTM_EWORKSPACE;
  if (e != TTM_OK && enqueued) (void)hipStreamSynchronize(st);
  return e;
}

// Sizes of the reverse mode: the product's workspace, its record, the
// largest core and SVD matrix (doubles), and the output capacity.
int vjp_sizes(const ttm_tt *A, const ttm_tt *B, int chi_out, const ttm_options *opt, size_t *fwd_ws,
              int64_t *tape_doubles, int64_t *max_core, int64_t *max_mn, int64_t *out_capacity) {
  int e = validate_pair(A, B);
  if (e) return e;
  if (chi_out < 1) return TTM_EINVAL;
  Options o;
  e = resolve_options(opt, chi_out, o);
  if (e) return e;
  if (o.gauge != TTM_GAUGE_MOVING || o.svd_mode != TTM_SVD_JACOBI) return TTM_EUNSUPPORTED;
  Plan pl;
  e = make_plan(A, B, chi_out, o, pl);
  if (e) return e;
  *fwd_ws = pl.ws_bytes;
  *tape_doubles = pl.tape + 64 * (int64_t)(8 * pl.n * pl.n + 16);  // per-entry alignment slack
  *max_core = pl.max_core;
  *max_mn = pl.max_mn;
  *out_capacity = pl.out_capacity;
  return TTM_OK;
}

namespace {

int run_ttm(const ttm_tt *A, const ttm_tt *B, int chi_out, double tol, ttm_tt_out *C, void *ws,
            size_t ws_bytes, hipStream_t st, const Options &o, ttm_stats *stats) {
  bool enqueued = false;
  const int e = run_ttm_impl(A, B, chi_out, tol, C, ws, ws_bytes, st, o, stats, enqueued);
  // On an error after work was enqueued, drain the stream so the caller may
  // release the workspace as soon as the call returns.
  if (e != TTM_OK && enqueued) (void)hipStreamSynchronize(st);
  return e;
}


// ====================================================================== conventional
// Single-site variational fit (Sec. II.A): C ~ A * B with bonds capped at
// chi_out, never forming the chi_A chi_B Kronecker carriages of
// Eq. (carriageXi).  Per site the optimal core is the projection
//   C_i[c, s, c'] = sum L[c, a, b] A_i[a, s, a'] B_i[b, s, b'] R[c', a', b'],
// contracted as (L B) then A over the shared physical index s, then R:
// chi^4 work, chi^3 environments.  Reading of the unstated details: seeded
// initial guess (counter-based SplitMix64), left-to-right then right-to-left
// sweeps, stop when the centre's norm changes by at most tol (relative)
// between two full sweeps, or after max_sweeps.

struct ConvPlan {
  int n = 0;
  std::vector<int> phys;
  std::vector<Shape> a, b, c;   // c: initial bonds (structural, capped at chi_out)
  std::vector<int64_t> lsz, rsz; // environment sizes (doubles)
  int64_t tmax = 1, core_max = 1, qr_max = 1, rmax = 1;
  int64_t out_capacity = 0;
  size_t ws_bytes = 0;
};

int make_conv_plan(const ttm_tt *A, const ttm_tt *B, int chi_out, ConvPlan &pl) {
  const int n = A->n_sites;
  pl.n = n;
  pl.phys.assign(A->phys, A->phys + n);
  pl.a.resize(n); pl.b.resize(n); pl.c.resize(n);
  std::vector<int> cb(n + 1, 1);
  for (int i = 1; i < n; ++i) cb[i] = (int)std::min<int64_t>(product_bound(pl.phys, i), chi_out);
  for (int i = 0; i < n; ++i) {
    pl.a[i] = {A->bonds[i], A->phys[i], A->bonds[i + 1]};
    pl.b[i] = {B->bonds[i], B->phys[i], B->bonds[i + 1]};
    pl.c[i] = {cb[i], pl.phys[i], cb[i + 1]};
    pl.core_max = std::max(pl.core_max, pl.c[i].size());
    pl.out_capacity += pl.c[i].size();
  }
  pl.lsz.assign(n + 1, 1);
  pl.rsz.assign(n + 1, 1);
  for (int i = 0; i <= n; ++i) {
    const int64_t e = (int64_t)cb[i] * A->bonds[i] * B->bonds[i];
    if (e > kMaxEntries) return TTM_EINVAL;
    pl.lsz[i] = e;
    pl.rsz[i] = e;
  }
  for (int i = 0; i < n; ++i) {
    const int64_t cl = cb[i], cr = cb[i + 1], al = pl.a[i].rl, ar = pl.a[i].rr, br = pl.b[i].rr,
                  d = pl.phys[i];
    pl.tmax = std::max(pl.tmax, std::max(cl * al * d * br, cl * d * ar * br));
    if (!unfolding_ok(cl * d, cr) || !unfolding_ok(d * cr, cl)) return TTM_EINVAL;
    pl.qr_max = std::max<int64_t>(pl.qr_max, (int64_t)qr_scratch_doubles((int)(cl * d), (int)cr));
    pl.qr_max = std::max<int64_t>(pl.qr_max, (int64_t)qr_scratch_doubles((int)(d * cr), (int)cl));
    pl.rmax = std::max(pl.rmax, std::max(cl * d, cr) * std::max(cl, cr));
  }
  size_t bytes = 0;
  for (int i = 0; i <= n; ++i) bytes += align_up((size_t)pl.lsz[i] * 8) + align_up((size_t)pl.rsz[i] * 8);
  bytes += 2 * align_up((size_t)pl.tmax * 8);
  bytes += (size_t)(n + 3) * align_up((size_t)pl.core_max * 8);
  bytes += align_up((size_t)pl.qr_max * 8) + align_up((size_t)pl.rmax * 8) + 256;
  pl.ws_bytes = bytes;
  if (pl.tmax > ((int64_t)1 << 36)) return TTM_EINVAL;
  return TTM_OK;
}

struct ConvRunner {
  hipStream_t st;
  KernelTimer timer;
  int err = TTM_OK;
  double flops = 0.0;
  int n_qr = 0;
  bool hip(hipError_t e) {
    if (e != hipSuccess && err == TTM_OK) {
      err = TTM_EHIP;
      note_hip_error(e, "the conventional variational product");
    }
    return e == hipSuccess;
  }
  void gemm(const GemmArgs &g) {
    Timed tm(&timer, KC_GEMM, st);
    hip(launch_gemm(g, st));
    flops += 2.0 * g.M * (double)g.N * g.K * g.batch;
  }
};

int run_conventional_impl(const ttm_tt *A, const ttm_tt *B, int chi_out, double tol, ttm_tt_out *C,
                          void *ws, size_t ws_bytes, hipStream_t st, const Options &o,
                          ttm_stats *stats, bool &enqueued) {
  ConvPlan pl;
  int e = make_conv_plan(A, B, chi_out, pl);
  if (e) return e;
  if (!ws || ws_bytes < pl.ws_bytes) return TTM_EWORKSPACE;
  if (!C || !C->bonds || !C->offsets || !C->data) return TTM_EINVAL;
  if (C->capacity < pl.out_capacity) return TTM_ECAPACITY;
  const int n = pl.n;
  ConvRunner R;
  R.st = st;
  R.timer.on = o.profile != 0;
  enqueued = true;

  char *base = static_cast<char *>(ws);
  size_t off = 0;
  auto carve = [&](int64_t nd) {
    double *p = reinterpret_cast<double *>(base + off);
    off += align_up((size_t)nd * 8);
    return p;
  };
  std::vector<double *> L(n + 1), Rv(n + 1);
  for (int i = 0; i <= n; ++i) L[i] = carve(pl.lsz[i]);
  for (int i = 0; i <= n; ++i) Rv[i] = carve(pl.rsz[i]);
  double *T1 = carve(pl.tmax), *T2 = carve(pl.tmax);
  std::vector<double *> slots;
  for (int i = 0; i < n + 3; ++i) slots.push_back(carve(pl.core_max));
  double *qrs = carve(pl.qr_max), *rbuf = carve(pl.rmax);
  double *scal = carve(32);
  std::vector<double *> freeq(slots.begin() + n, slots.end());
  auto take = [&]() { double *p = freeq.back(); freeq.pop_back(); return p; };
  auto give = [&](double *p) { freeq.push_back(p); };

  const double *Ad = static_cast<const double *>(A->data);
  const double *Bd = static_cast<const double *>(B->data);
  std::vector<const double *> Ap(n), Bp(n);
  for (int i = 0; i < n; ++i) {
    Ap[i] = Ad + A->offsets[i];
    Bp[i] = Bd + B->offsets[i];
  }
  // initial guess
  std::vector<double *> Cp(slots.begin(), slots.begin() + n);
  std::vector<Shape> cs = pl.c;
  {
    Timed tm(&R.timer, KC_OTHER, st);
    int64_t start = 0;
    for (int i = 0; i < n; ++i) {
      R.hip(launch_splitmix_fill(Cp[i], cs[i].size(), o.seed, start, st));
      start += cs[i].size();
    }
    R.hip(launch_fill(L[0], 1.0, 1, st));
    R.hip(launch_fill(Rv[n], 1.0, 1, st));
  }

  // LQ of core i (rows: left bond), the R factor pushed into core i-1.
  auto lq_left = [&](int i, bool push) {
    const Shape s = cs[i];
    const int m = s.d * s.rr, nn = s.rl, k = std::min(m, nn);
    double *q = take();
    {
      Timed tm(&R.timer, KC_QR, st);
      R.hip(launch_qr(Cp[i], m, nn, 1, m, q, rbuf, qrs, st));
    }
    double *qt = take();
    {
      Timed tm(&R.timer, KC_OTHER, st);
      R.hip(launch_transpose(qt, q, m, k, st));
    }
    give(q);
    ++R.n_qr;
    R.flops += 4.0 * m * (double)nn * nn;
    if (push) {
      const Shape p = cs[i - 1];
      double *np_ = take();
      GemmArgs g;
      g.M = p.rl * p.d; g.N = k; g.K = nn;
      g.A = Cp[i - 1]; g.a_rs = p.rr; g.a_cs = 1;
      g.B = rbuf; g.b_rs = 1; g.b_cs = nn;  // R^T
      g.C = np_; g.c_rs1 = k; g.c_cs1 = 1;
      R.gemm(g);
      give(Cp[i - 1]);
      Cp[i - 1] = np_;
      cs[i - 1].rr = k;
    }
    give(Cp[i]);
    Cp[i] = qt;
    cs[i].rl = k;
  };

  // right environment R_i from core i and R_{i+1}
  auto right_env = [&](int i) {
    const int64_t cl = cs[i].rl, d = cs[i].d, cr = cs[i].rr;
    const int64_t al = pl.a[i].rl, ar = pl.a[i].rr, bl = pl.b[i].rl, br = pl.b[i].rr;
    R.gemm(gemm_rowmajor((int)(cl * d), (int)(ar * br), (int)cr, Cp[i], cr, Rv[i + 1], ar * br, T1, ar * br));
    for (int s = 0; s < d; ++s) {
      GemmArgs g;
      g.M = (int)al; g.N = (int)br; g.K = (int)ar; g.batch = (int)cl;
      g.A = Ap[i] + s * ar; g.a_rs = d * ar; g.a_cs = 1; g.a_bs = 0;
      g.B = T1 + s * ar * br; g.b_rs = br; g.b_cs = 1; g.b_bs = d * ar * br;
      g.C = T2 + s * br; g.c_rs1 = d * br; g.c_cs1 = 1; g.c_bs = al * d * br;
      R.gemm(g);
    }
    GemmArgs g;
    g.M = (int)al; g.N = (int)bl; g.K = (int)(d * br); g.batch = (int)cl;
    g.A = T2; g.a_rs = d * br; g.a_cs = 1; g.a_bs = al * d * br;
    g.B = Bp[i]; g.b_rs = 1; g.b_cs = d * br; g.b_bs = 0;
    g.C = Rv[i]; g.c_rs1 = bl; g.c_cs1 = 1; g.c_bs = al * bl;
    R.gemm(g);
  };

  // local optimum at site i from L_i and R_{i+1}; leaves T2 = (L B) A
  auto local = [&](int i, double *out) {
    const int64_t cl = cs[i].rl, d = pl.phys[i], cr = cs[i].rr;
    const int64_t al = pl.a[i].rl, ar = pl.a[i].rr, bl = pl.b[i].rl, br = pl.b[i].rr;
    R.gemm(gemm_rowmajor((int)(cl * al), (int)(d * br), (int)bl, L[i], bl, Bp[i], d * br, T1, d * br));
    for (int s = 0; s < d; ++s) {
      GemmArgs g;
      g.M = (int)ar; g.N = (int)br; g.K = (int)al; g.batch = (int)cl;
      g.A = Ap[i] + s * ar; g.a_rs = 1; g.a_cs = d * ar; g.a_bs = 0;
      g.B = T1 + s * br; g.b_rs = d * br; g.b_cs = 1; g.b_bs = al * d * br;
      g.C = T2 + s * ar * br; g.c_rs1 = br; g.c_cs1 = 1; g.c_bs = d * ar * br;
      R.gemm(g);
    }
    GemmArgs g;
    g.M = (int)(cl * d); g.N = (int)cr; g.K = (int)(ar * br);
    g.A = T2; g.a_rs = ar * br; g.a_cs = 1;
    g.B = Rv[i + 1]; g.b_rs = 1; g.b_cs = ar * br;
    g.C = out; g.c_rs1 = cr; g.c_cs1 = 1;
    R.gemm(g);
  };

  // right-orthogonalise the initial guess and build the right environments
  for (int i = n - 1; i >= 1 && !R.err; --i) lq_left(i, true);
  for (int i = n - 1; i >= 1 && !R.err; --i) right_env(i);

  int sweeps = 0;
  double prev = -1.0, nrm = 0.0;
  for (int sw = 0; sw < o.max_sweeps && !R.err; ++sw) {
    ++sweeps;
    for (int i = 0; i < n && !R.err; ++i) {
      double *cn = take();
      local(i, cn);
      give(Cp[i]);
      Cp[i] = cn;
      if (i < n - 1) {
        const Shape s = cs[i];
        const int m = s.rl * s.d, nn = s.rr, k = std::min(m, nn);
        double *q = take();
        {
          Timed tm(&R.timer, KC_QR, st);
          R.hip(launch_qr(Cp[i], m, nn, nn, 1, q, rbuf, qrs, st));
        }
        ++R.n_qr;
        R.flops += 4.0 * m * (double)nn * nn;
        give(Cp[i]);
        Cp[i] = q;
        cs[i].rr = k;
        cs[i + 1].rl = k;
        // L_{i+1}[c', a', b'] = sum_{c,s} Q[c,s,c'] T2[c,s,a',b']
        const int64_t ar = pl.a[i].rr, br = pl.b[i].rr;
        GemmArgs g;
        g.M = k; g.N = (int)(ar * br); g.K = m;
        g.A = Cp[i]; g.a_rs = 1; g.a_cs = k;
        g.B = T2; g.b_rs = ar * br; g.b_cs = 1;
        g.C = L[i + 1]; g.c_rs1 = ar * br; g.c_cs1 = 1;
        R.gemm(g);
      }
    }
    for (int i = n - 1; i >= 0 && !R.err; --i) {
      double *cn = take();
      local(i, cn);
      give(Cp[i]);
      Cp[i] = cn;
      if (i > 0) {
        lq_left(i, false);
        cs[i - 1].rr = cs[i].rl;
        right_env(i);
      }
    }
    {
      Timed tm(&R.timer, KC_OTHER, st);
      R.hip(launch_sumsq(Cp[0], cs[0].size(), scal, st));
    }
    double h = 0.0;
    R.hip(hipMemcpyAsync(&h, scal, sizeof(double), hipMemcpyDeviceToHost, st));
    R.hip(hipStreamSynchronize(st));
    if (R.timer.on) R.timer.collect();
    if (R.err) break;
    if (!std::isfinite(h)) return TTM_ENONFINITE;
    nrm = sqrt(h);
    if (prev >= 0.0 && fabs(nrm - prev) <= tol * nrm) break;
    prev = nrm;
  }
  if (R.err) return R.err;
  int64_t pos = 0;
  double *Cd = static_cast<double *>(C->data);
  for (int i = 0; i < n; ++i) {
    C->offsets[i] = pos;
    C->bonds[i] = cs[i].rl;
    Timed tm(&R.timer, KC_OTHER, st);
    R.hip(launch_copy(Cd + pos, Cp[i], cs[i].size(), st));
    pos += cs[i].size();
  }
  C->bonds[n] = cs[n - 1].rr;
  R.hip(hipStreamSynchronize(st));
  if (R.timer.on) R.timer.collect();
  if (R.err) return R.err;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    int mb = 1;
    for (int i = 0; i < n; ++i) mb = std::max(mb, cs[i].rr);
    stats->max_bond = mb;
    stats->n_qr = R.n_qr;
    stats->sweeps = sweeps;
    stats->model_flops = R.flops;
    stats->peak_ws_bytes = pl.ws_bytes;
    for (int c = 0; c < KC_COUNT; ++c) {
      stats->kernel_ms[c] = R.timer.ms[c];
      stats->kernel_launches[c] = R.timer.launches[c];
    }
  }
  return TTM_OK;
}

int run_conventional(const ttm_tt *A, const ttm_tt *B, int chi_out, double tol, ttm_tt_out *C, void *ws,
                     size_t ws_bytes, hipStream_t st, const Options &o, ttm_stats *stats) {
  bool enqueued = false;
  const int e = run_conventional_impl(A, B, chi_out, tol, C, ws, ws_bytes, st, o, stats, enqueued);
  if (e != TTM_OK && enqueued) (void)hipStreamSynchronize(st);
  return e;
}

}  // namespace
}  // namespace ttm

// ====================================================================== C ABI
extern "C" {

void ttm_default_options(ttm_options *opt) {
  if (!opt) return;
  memset(opt, 0, sizeof(*opt));
  opt->chi_mid = -1;
  opt->final_round = 1;
  opt->max_sweeps = 10;
  opt->svd_max_sweeps = 40;
  opt->seed = 12345;
  opt->svd_mode = TTM_SVD_JACOBI;
  opt->rsvd_power = 10;
  opt->rsvd_tol = 2e-8;
}

const char *ttm_strerror(int code) {
  switch (code) {
    case TTM_OK: return "ok";
    case TTM_EINVAL: return "invalid argument";
    case TTM_ESHAPE: return "shape mismatch between the two trains or bad end bonds";
    case TTM_EWORKSPACE: return "workspace missing or too small";
    case TTM_ECAPACITY: return "output buffer too small";
    case TTM_ENOCONV: return "SVD did not converge";
    case TTM_ENONFINITE: return "NaN or Inf in the data";
    case TTM_EHIP: return "HIP runtime error";
    case TTM_EFORCED: return "forced rank list inconsistent with the schedule";
    case TTM_EUNSUPPORTED: return "unsupported dtype or option combination, or an SVD larger than the kernels take";
    default: return "unknown error";
  }
}

const char *ttm_version(void) { return "libttm 0.2 (gfx950, fp64)"; }

const char *ttm_last_error(void) { return ttm::last_error_text(); }

int ttm_query(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, const ttm_options *opt,
              size_t *ws_bytes, int64_t *out_capacity) {
  int e = ttm::validate_pair(A, B);
  if (e) return e;
  if (chi_out < 1) return TTM_EINVAL;
  ttm::Options o;
  e = ttm::resolve_options(opt, chi_out, o);
  if (e) return e;
  ttm::Plan pl;
  e = ttm::make_plan(A, B, chi_out, o, pl);
  if (e) return e;
  if (ws_bytes) *ws_bytes = pl.ws_bytes;
  if (out_capacity) *out_capacity = pl.out_capacity;
  return TTM_OK;
}

int ttm_multiply_ex(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol, ttm_tt_out *C,
                    void *ws, size_t ws_bytes, void *stream, const ttm_options *opt,
                    ttm_stats *stats) {
  ttm::clear_last_error();
  int e = ttm::validate_pair(A, B);
  if (e) return e;
  if (chi_out < 1) return TTM_EINVAL;
  if (!(tol >= 0.0) || !isfinite(tol)) return TTM_EINVAL;
  ttm::Options o;
  e = ttm::resolve_options(opt, chi_out, o);
  if (e) return e;
  return ttm::run_ttm(A, B, chi_out, tol, C, ws, ws_bytes, static_cast<hipStream_t>(stream), o, stats);
}

int ttm_multiply(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol, ttm_tt_out *C,
                 void *ws, size_t ws_bytes, void *stream) {
  return ttm_multiply_ex(A, B, chi_out, tol, C, ws, ws_bytes, stream, nullptr, nullptr);
}

int conventional_query(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, const ttm_options *opt,
                       size_t *ws_bytes, int64_t *out_capacity) {
  int e = ttm::validate_pair(A, B);
  if (e) return e;
  if (chi_out < 1) return TTM_EINVAL;
  ttm::Options o;
  e = ttm::resolve_options(opt, chi_out, o);
  if (e) return e;
  ttm::ConvPlan pl;
  e = ttm::make_conv_plan(A, B, chi_out, pl);
  if (e) return e;
  if (ws_bytes) *ws_bytes = pl.ws_bytes;
  if (out_capacity) *out_capacity = pl.out_capacity;
  return TTM_OK;
}

int conventional_multiply_ex(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol,
                             ttm_tt_out *C, void *ws, size_t ws_bytes, void *stream,
                             const ttm_options *opt, ttm_stats *stats) {
  ttm::clear_last_error();
  int e = ttm::validate_pair(A, B);
  if (e) return e;
  if (chi_out < 1) return TTM_EINVAL;
  if (!(tol >= 0.0) || !isfinite(tol)) return TTM_EINVAL;
  ttm::Options o;
  e = ttm::resolve_options(opt, chi_out, o);
  if (e) return e;
  return ttm::run_conventional(A, B, chi_out, tol, C, ws, ws_bytes, static_cast<hipStream_t>(stream), o,
                               stats);
}

int conventional_multiply(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol,
                          ttm_tt_out *C, void *ws, size_t ws_bytes, void *stream) {
  return conventional_multiply_ex(A, B, chi_out, tol, C, ws, ws_bytes, stream, nullptr, nullptr);
}

}  // extern "C"
