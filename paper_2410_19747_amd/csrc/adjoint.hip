// Gradient of L = <W, A*B> with respect to the cores of A and B by
// three-train environments.  Every contraction is one strided (batched) GEMM
// on the matrix cores; the strides and split output mappings below put each
// intermediate in the layout the next contraction reads with unit stride.
//
// Index names per site k: w, a, b are the left bonds of W, A, B (sizes rw,
// ra, rb), w', a', b' the right bonds (rw2, ra2, rb2), s the physical index
// (d).  Core X_k[x][s][x'] is row-major.  Environments are [w][a][b]
// row-major.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ttm_internal.h"

namespace ttm {
namespace {

size_t r32(size_t n) { return (n + 31) & ~(size_t)31; }
constexpr int64_t kSplitSlices = 16;  // split-K scratch: up to 16 partial outputs per contraction

int check_train(const ttm_tt *t) {
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

int check_triple(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B) {
  int e = check_train(W);
  if (!e) e = check_train(A);
  if (!e) e = check_train(B);
  if (e) return e;
  if (A->n_sites != W->n_sites || B->n_sites != W->n_sites) return TTM_ESHAPE;
  for (int i = 0; i < W->n_sites; ++i)
    if (A->phys[i] != W->phys[i] || B->phys[i] != W->phys[i]) return TTM_ESHAPE;
  return TTM_OK;
}

struct GradPlan {
  int n = 0;
  // Right environments.  stride 1: F_k at env_off[k] (doubles), all kept.
  // stride s >= 2: the checkpoints F_k with (N - k) % s == 0 in slots
  // (N - k) / s, every other F_k in slot nck + (c - k - 1) of the segment
  // buffer, c the checkpoint above k; slots of env_max doubles.
  int stride = 1, nck = 0;
  std::vector<int64_t> env_off;
  int64_t env_total = 0, env_max = 0;
  int64_t x_max = 0;  // T1 (left sweep) / U1 (right sweep)
  int64_t y_max = 0;  // T2 / U2
  int64_t v_max = 0;  // V
  int64_t part = 0;   // split-K partial tiles of the skinny contractions
  size_t ws_doubles = 0;
  bool fits = true;
};

GradPlan make_grad_plan(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int stride) {
  GradPlan p;
  const int n = W->n_sites;
  p.n = n;
  if (stride == 0) stride = std::max(2, (int)std::ceil(std::sqrt((double)n)));
  p.stride = std::max(1, std::min(stride, std::max(n, 1)));
  p.env_off.resize(n + 1);
  // GEMM extents are ints and every buffer holds at most 2^36 doubles (beyond
  // any device memory); each limit is checked before the products it bounds,
  // so no size below can overflow.  Bonds are at most 2^20, dimensions 2^16.
  const int64_t lim = (int64_t)1 << 30, max_entries = (int64_t)1 << 36;
  auto env = [&](int k) { return (int64_t)W->bonds[k] * A->bonds[k] * B->bonds[k]; };
  for (int k = 0; k <= n; ++k) {
    if (env(k) > max_entries) {
      p.fits = false;
      return p;
    }
    p.env_off[k] = p.env_total;
    p.env_total += (int64_t)r32(env(k));
    p.env_max = std::max(p.env_max, env(k));
  }
  for (int k = 0; k < n; ++k) {
    const int64_t d = W->phys[k], rw = W->bonds[k], rw2 = W->bonds[k + 1];
    const int64_t ra = A->bonds[k], ra2 = A->bonds[k + 1], rb = B->bonds[k], rb2 = B->bonds[k + 1];
    if (ra * rb > lim || rw2 * ra2 > lim || d * rw2 > lim || ra2 * rb2 > lim || rw * ra > lim ||
        rw * d > lim || rb * d > lim || rb * rw2 > lim || rw * rb2 > lim || d * rb2 > lim) {
      p.fits = false;
      return p;
    }
    // Each product below is two of the checked pairs, so at most 2^60.
    p.x_max = std::max({p.x_max, (d * rw2) * (ra * rb), (rw * d) * (ra2 * rb2)});
    p.y_max = std::max({p.y_max, (rb * d) * (rw2 * ra2), (rw * ra) * (d * rb2)});
    p.v_max = std::max(p.v_max, (rb * d) * (rw2 * ra2));
    p.part = std::max({p.part, d * ra * ra2, d * rb * rb2, (rw2 * ra2) * rb2, (rw * ra) * rb});
    if (p.x_max > max_entries || p.y_max > max_entries || p.part > max_entries) {
      p.fits = false;
      return p;
    }
  }
  p.part *= kSplitSlices;
  if (p.stride > 1) {
    p.nck = (n - 1) / p.stride + 1;  // F_N, F_{N-s}, ... down to F_1 or above
    p.env_total = (int64_t)(p.nck + p.stride - 1) * r32(p.env_max);
  }
  p.ws_doubles = (size_t)p.env_total + 2 * r32(p.env_max) + r32(p.x_max) + r32(p.y_max) + r32(p.v_max) +
                 r32(p.part) + 32;
  return p;
}

const double *core(const ttm_tt *t, int k) { return static_cast<const double *>(t->data) + t->offsets[k]; }

GemmArgs strided(int M, int N, int K, int batch, const double *Am, int64_t a_rs, int64_t a_cs, int64_t a_bs,
                 const double *Bm, int64_t b_rs, int64_t b_cs, int64_t b_bs, double *C, int64_t c_bs,
                 int c_rdiv, int64_t c_rs1, int64_t c_rs0, int c_cdiv, int64_t c_cs1, int64_t c_cs0, int prec) {
  GemmArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.batch = batch;
  g.A = Am;
  g.a_rs = a_rs;
  g.a_cs = a_cs;
  g.a_bs = a_bs;
  g.B = Bm;
  g.b_rs = b_rs;
  g.b_cs = b_cs;
  g.b_bs = b_bs;
  g.C = C;
  g.c_bs = c_bs;
  g.c_rdiv = c_rdiv;
  g.c_rs1 = c_rs1;
  g.c_rs0 = c_rs0;
  g.c_cdiv = c_cdiv;
  g.c_cs1 = c_cs1;
  g.c_cs0 = c_cs0;
  g.prec = prec;
  return g;
}

}  // namespace

int inner_grad_query(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int stride, size_t *ws_bytes) {
  const int e = check_triple(W, A, B);
  if (e) return e;
  if (stride < 0) return TTM_EINVAL;
  const GradPlan p = make_grad_plan(W, A, B, stride);
  if (!p.fits) return TTM_EINVAL;
  if (ws_bytes) *ws_bytes = p.ws_doubles * sizeof(double);
  return TTM_OK;
}

int inner_grad(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int prec, double *value, double *dA,
               double *dB, int stride, void *ws, size_t ws_bytes, hipStream_t st) {
  int e = check_triple(W, A, B);
  if (e) return e;
  if (!value || stride < 0) return TTM_EINVAL;
  if (prec < TTM_PREC_F64 || prec > TTM_PREC_BF16X3) return TTM_EINVAL;
  const GradPlan p = make_grad_plan(W, A, B, stride);
  if (!p.fits) return TTM_EINVAL;
  if (!ws || ws_bytes < p.ws_doubles * sizeof(double)) return TTM_EWORKSPACE;
  const int gp = prec == TTM_PREC_F32 ? GEMM_F32 : prec == TTM_PREC_BF16 ? GEMM_BF16
                 : prec == TTM_PREC_BF16X3 ? GEMM_BF16X3 : GEMM_F64;
  double *base = static_cast<double *>(ws);
  double *R = base;  // right environments
  double *Lc = R + p.env_total;
  double *Ln = Lc + r32(p.env_max);
  double *X = Ln + r32(p.env_max);
  double *Y = X + r32(p.x_max);
  double *V = Y + r32(p.y_max);
  double *P = V + r32(p.v_max);  // split-K partial tiles
  const bool grads = dA || dB;
  auto gemm = [&](GemmArgs g) {
    g.part = P;
    g.part_doubles = p.part;
    return launch_gemm(g, st);
  };
  const int n = p.n;
  auto fail = [&](hipError_t h) {
    note_hip_error(h, "the environment sweeps of ttm_inner_grad");
    (void)hipStreamSynchronize(st);
    return TTM_EHIP;
  };
  hipError_t h;
  // Right environments F_N .. F_1 (F_0 is not needed), only for gradients.
  const int s = p.stride;
  const int64_t slot = r32(p.env_max);
  auto is_ck = [&](int k) { return (n - k) % s == 0; };
  auto env_at = [&](int k) -> double * {
    if (s == 1) return R + p.env_off[k];
    if (is_ck(k)) return R + (int64_t)((n - k) / s) * slot;
    const int c = n - ((n - k) / s) * s;  // the checkpoint above k
    return R + (int64_t)(p.nck + (c - k - 1)) * slot;
  };
  // F_k from F_{k+1} (three products)
  auto right_step = [&](int k) -> hipError_t {
    const int d = W->phys[k], rw = W->bonds[k], rw2 = W->bonds[k + 1];
    const int ra = A->bonds[k], ra2 = A->bonds[k + 1], rb = B->bonds[k], rb2 = B->bonds[k + 1];
    const double *Rn = env_at(k + 1);
    // U1[s][a'][w][b'] = sum_w' W[w,s,w'] F_{k+1}[w',a',b']  (rows w*d+s, columns a'*rb2+b')
    GemmArgs g1 = strided(rw * d, ra2 * rb2, rw2, 1, core(W, k), rw2, 1, 0, Rn, (int64_t)ra2 * rb2, 1, 0, X, 0,
                          d, rb2, (int64_t)ra2 * rw * rb2, rb2, (int64_t)rw * rb2, 1, gp);
    // U2[w][a][s][b'] = sum_a' A[a,s,a'] U1[s][a'][w][b']  (batch s; rows a, columns w*rb2+b')
    GemmArgs g2 = strided(ra, rw * rb2, ra2, d, core(A, k), (int64_t)d * ra2, 1, ra2, X, (int64_t)rw * rb2, 1,
                          (int64_t)ra2 * rw * rb2, Y, rb2, 1, (int64_t)d * rb2, 0, rb2,
                          (int64_t)ra * d * rb2, 1, gp);
    // F_k[w][a][b] = sum_{s,b'} U2[w][a][s][b'] B[b,s,b']  (rows w*ra+a, K = s*rb2+b')
    GemmArgs g3 = strided(rw * ra, rb, d * rb2, 1, Y, (int64_t)d * rb2, 1, 0, core(B, k), 1, (int64_t)d * rb2, 0,
                          env_at(k), 0, 1, rb, 0, 1, 1, 0, gp);
    hipError_t h1;
    if ((h1 = gemm(g1)) != hipSuccess || (h1 = gemm(g2)) != hipSuccess) return h1;
    return gemm(g3);
  };
  // With checkpoints the sweep leaves the lowest segment (F_1 upwards) in the
  // segment buffer; the left sweep recomputes each higher segment from its
  // checkpoint when it reaches it (same products on the same inputs, so the
  // same values).
  int seg_loaded = -1;  // checkpoint above the segment the buffer holds
  if (grads) {
    if ((h = launch_fill(env_at(n), 1.0, 1, st)) != hipSuccess) return fail(h);
    for (int k = n - 1; k >= 1; --k)
      if ((h = right_step(k)) != hipSuccess) return fail(h);
    if (s > 1 && n > 1 && !is_ck(1)) seg_loaded = n - ((n - 1) / s) * s;
  }
  // Left sweep: E_0 = 1; at each site the gradients, then E_{k+1}.
  if ((h = launch_fill(Lc, 1.0, 1, st)) != hipSuccess) return fail(h);
  for (int k = 0; k < n; ++k) {
    // F_{k+1} in a segment the buffer does not hold: F_{c-1} .. F_{k+1} from
    // the checkpoint F_c above (before T1 and T2, whose buffers it uses)
    if (grads && s > 1 && !is_ck(k + 1)) {
      const int c = n - ((n - k - 1) / s) * s;
      if (c != seg_loaded) {
        for (int j = c - 1; j >= k + 1; --j)
          if ((h = right_step(j)) != hipSuccess) return fail(h);
        seg_loaded = c;
      }
    }
    const int d = W->phys[k], rw = W->bonds[k], rw2 = W->bonds[k + 1];
    const int ra = A->bonds[k], ra2 = A->bonds[k + 1], rb = B->bonds[k], rb2 = B->bonds[k + 1];
    // T1[s][a][b][w'] = sum_w E_k[w,a,b] W[w,s,w']  (rows a*rb+b, columns s*rw2+w')
    GemmArgs t1 = strided(ra * rb, d * rw2, rw, 1, Lc, 1, (int64_t)ra * rb, 0, core(W, k), (int64_t)d * rw2, 1, 0,
                          X, 0, 1, rw2, 0, rw2, (int64_t)ra * rb * rw2, 1, gp);
    // T2[b][s][w'][a'] = sum_a T1[s][a][b][w'] A[a,s,a']  (batch s; rows b*rw2+w', columns a')
    GemmArgs t2 = strided(rb * rw2, ra2, ra, d, X, 1, (int64_t)rb * rw2, (int64_t)ra * rb * rw2, core(A, k),
                          (int64_t)d * ra2, 1, ra2, Y, (int64_t)rw2 * ra2, rw2, (int64_t)d * rw2 * ra2, ra2, 1, 1,
                          0, gp);
    if ((h = gemm(t1)) != hipSuccess || (h = gemm(t2)) != hipSuccess) return fail(h);
    if (grads) {
      const double *Rn = env_at(k + 1);
      if (dB) {
        // dB_k[b,s,b'] = sum_{w',a'} T2[b][s][w'][a'] F_{k+1}[w'][a'][b']  (rows b*d+s)
        GemmArgs gb = strided(rb * d, rb2, rw2 * ra2, 1, Y, (int64_t)rw2 * ra2, 1, 0, Rn, rb2, 1, 0,
                              dB + B->offsets[k], 0, 1, rb2, 0, 1, 1, 0, gp);
        if ((h = gemm(gb)) != hipSuccess) return fail(h);
      }
      if (dA) {
        // V[s][b][w'][a'] = sum_b' B[b,s,b'] F_{k+1}[w'][a'][b']  (batch s; rows b, columns w'*ra2+a')
        GemmArgs gv = strided(rb, rw2 * ra2, rb2, d, core(B, k), (int64_t)d * rb2, 1, rb2, Rn, 1, rb2, 0, V,
                              (int64_t)rb * rw2 * ra2, 1, (int64_t)rw2 * ra2, 0, 1, 1, 0, gp);
        // dA_k[a,s,a'] = sum_{b,w'} T1[s][a][b][w'] V[s][b][w'][a']  (batch s)
        GemmArgs ga = strided(ra, ra2, rb * rw2, d, X, (int64_t)rb * rw2, 1, (int64_t)ra * rb * rw2, V, ra2, 1,
                              (int64_t)rb * rw2 * ra2, dA + A->offsets[k], ra2, 1, (int64_t)d * ra2, 0, 1, 1,
                              0, gp);
        if ((h = gemm(gv)) != hipSuccess || (h = gemm(ga)) != hipSuccess) return fail(h);
      }
    }
    // E_{k+1}[w'][a'][b'] = sum_{b,s} T2[b][s][w'][a'] B[b,s,b']  (rows w'*ra2+a', K = b*d+s)
    GemmArgs t3 = strided(rw2 * ra2, rb2, rb * d, 1, Y, 1, (int64_t)rw2 * ra2, 0, core(B, k), rb2, 1, 0, Ln, 0, 1,
                          rb2, 0, 1, 1, 0, gp);
    if ((h = gemm(t3)) != hipSuccess) return fail(h);
    std::swap(Lc, Ln);
  }
  if ((h = hipMemcpyAsync(value, Lc, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess) return fail(h);
  if ((h = hipStreamSynchronize(st)) != hipSuccess) {
    note_hip_error(h, "the synchronisation at the end of ttm_inner_grad");
    return TTM_EHIP;
  }
  if (!isfinite(*value)) {
    set_last_error("the inner product <W, A*B> is not finite");
    return TTM_ENONFINITE;
  }
  return TTM_OK;
}

}  // namespace ttm

extern "C" int ttm_inner_grad_query(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, size_t *ws_bytes) {
  return ttm::inner_grad_query(W, A, B, 1, ws_bytes);
}

extern "C" int ttm_inner_grad(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int32_t contract_precision,
                              double *value, double *dA, double *dB, void *ws, size_t ws_bytes, void *stream) {
  ttm::clear_last_error();
  return ttm::inner_grad(W, A, B, contract_precision, value, dA, dB, 1, ws, ws_bytes,
                         static_cast<hipStream_t>(stream));
}

extern "C" int ttm_inner_grad_query_ex(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int32_t env_stride,
                                       size_t *ws_bytes) {
  return ttm::inner_grad_query(W, A, B, env_stride, ws_bytes);
}

extern "C" int ttm_inner_grad_ex(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int32_t contract_precision,
                                 double *value, double *dA, double *dB, int32_t env_stride, void *ws,
                                 size_t ws_bytes, void *stream) {
  ttm::clear_last_error();
  return ttm::inner_grad(W, A, B, contract_precision, value, dA, dB, env_stride, ws, ws_bytes,
                         static_cast<hipStream_t>(stream));
}
