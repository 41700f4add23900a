// Truncated SVD driver for the swap and rounding steps: column ordering,
// two Householder QRs as preconditioner, one-sided Jacobi on R2^T, rank rule
// and write-out (the steps are listed with svd_oside in ttm_internal.h).
#include <math.h>
#include <stdio.h>

#include <algorithm>

#include "ttm_internal.h"

namespace ttm {
namespace {
constexpr double kUnitRoundoff = 2.220446049250313e-16;
constexpr int kPanel = 16;  // QR panel width (T factors of 16 x 16 per panel)

size_t r32(size_t n) { return (n + 31) & ~(size_t)31; }

struct SvdBufs {
  double *Xt = nullptr;    // no x np: X = Y^T; later R1^T (np x k), then U_r (no x r)
  double *S = nullptr;     // no x np: ordered copy of X, factored in place (Q1, R1)
  double *qr = nullptr;    // QR scratch (both factorisations)
  double *Tall = nullptr;  // T factors of the first QR
  double *xnorm = nullptr; // np column norms of X
  int *perm1 = nullptr;    // np: ordered position -> column of X
  JacobiBufs jb;
};

size_t qr_ws(const SvdPlan &p) {
  return std::max({qr_inplace_scratch_doubles(p.no, p.np), qr_inplace_scratch_doubles(p.np, p.k),
                   qr_apply_q_scratch_doubles(p.no, p.k)});
}

SvdBufs carve(const SvdPlan &p, double *base) {
  SvdBufs b;
  double *q = base;
  auto adv = [&](size_t nd) {
    double *x = q;
    q += r32(nd);
    return x;
  };
  const JacobiPlan &jp = p.jp;
  b.Xt = adv((size_t)p.np * p.no);
  b.S = adv((size_t)p.np * p.no);
  b.qr = adv(qr_ws(p));
  b.Tall = adv((size_t)((p.k + kPanel - 1) / kPanel) * kPanel * kPanel);
  b.xnorm = adv((size_t)p.np);
  b.perm1 = reinterpret_cast<int *>(adv((size_t)p.np));
  b.jb.W = adv((size_t)jp.L * jp.ncp);
  b.jb.Wt = adv((size_t)jp.L * jp.ncp);
  b.jb.part = adv((size_t)jp.pairs * jp.gsw * 4 * jp.bw * jp.bw);
  b.jb.conv = adv((size_t)jp.rounds * jp.pairs);
  b.jb.qbuf = adv((size_t)jp.pairs * 4 * jp.bw * jp.bw);
  b.jb.flag = reinterpret_cast<int *>(adv((size_t)jp.pairs));
  b.jb.sigma = adv((size_t)jp.ncp);
  b.jb.perm = reinterpret_cast<int *>(adv((size_t)jp.ncp));
  b.jb.result = adv(8);
  return b;
}

__global__ void sorted_sigma_kernel(const double *__restrict__ sigma, const int *__restrict__ perm, int n,
                                    double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = sigma[perm[t]];
}
}  // namespace

SvdPlan svd_plan(int np, int no, int force_bw) {
  SvdPlan p;
  p.np = np;
  p.no = no;
  p.k = std::min(np, no);
  p.jp = jacobi_plan(p.k, p.k, force_bw);
  return p;
}

size_t svd_ws_doubles(const SvdPlan &p) {
  const JacobiPlan &jp = p.jp;
  size_t n = 0;
  n += 2 * r32((size_t)p.np * p.no);
  n += r32(qr_ws(p));
  n += r32((size_t)((p.k + kPanel - 1) / kPanel) * kPanel * kPanel);
  n += 2 * r32((size_t)p.np);
  n += 2 * r32((size_t)jp.L * jp.ncp);
  n += r32((size_t)jp.pairs * jp.gsw * 4 * jp.bw * jp.bw);
  n += r32((size_t)jp.rounds * jp.pairs);
  n += r32((size_t)jp.pairs * 4 * jp.bw * jp.bw);
  n += r32((size_t)jp.pairs);
  n += 2 * r32((size_t)jp.ncp);
  n += r32(8);
  return n;
}

SvdResult svd_oside(const SvdPlan &p, const double *Y, double eps, int cap, int forced, int max_sweeps,
                    double *u, int u_layout, double *sigma_out, double *ws, hipStream_t s,
                    KernelTimer *timer, int trace, SvdAll *all, const double *full_total) {
  SvdResult out;
  SvdBufs b = carve(p, ws);
  const JacobiPlan &jp = p.jp;
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess) {
      out.err = TTM_EHIP;
      char what[96];
      snprintf(what, sizeof(what), "the truncated SVD of a %d x %d matrix", p.np, p.no);
      note_hip_error(e, what);
      if (trace) fprintf(stderr, "[ttm] HIP error %s (%s) in %s\n", hipGetErrorName(e), hipGetErrorString(e), what);
      return false;
    }
    return true;
  };
  auto sync = [&]() {
    if (!ok(hipStreamSynchronize(s))) return false;
    if (timer && timer->on) timer->collect();
    return true;
  };
  // 1. X = Y^T, its columns in decreasing norm order, ||Y||_F^2
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_transpose(b.Xt, Y, p.no, p.np, s))) return out;
    if (!ok(launch_column_norms(b.Xt, p.no, p.np, b.xnorm, s))) return out;
    if (!ok(launch_sort_desc(b.xnorm, p.np, b.perm1, s))) return out;
    if (!ok(launch_gather_columns(b.Xt, b.perm1, p.no, p.np, b.S, s))) return out;
    if (!ok(launch_frob_from_norms(b.xnorm, p.np, b.jb.result, s))) return out;
  }
  // 2. X P = Q1 R1, then R1^T = Q2 R2
  {
    Timed tm(timer, KC_QR, s);
    // No block column pivoting: it saves a few sweeps (about 2% at every
    // size measured) but its column moves cost more than they save once the
    // columns are presorted by norm.
    if (!ok(launch_qr_inplace(b.S, p.no, p.np, b.qr, nullptr, b.Tall, s))) return out;
  }
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_rt_from_qr(b.S, p.no, p.np, p.k, p.k, b.Xt, s))) return out;
  }
  {
    Timed tm(timer, KC_QR, s);
    if (!ok(launch_qr_inplace(b.Xt, p.np, p.k, b.qr, nullptr, nullptr, s))) return out;
  }
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_rt_from_qr(b.Xt, p.np, p.k, p.k, jp.ncp, b.jb.W, s))) return out;
  }
  // 3. Jacobi sweeps until the columns of W are orthogonal
  const double tol = sqrt((double)std::max(jp.L, 1)) * kUnitRoundoff;
  double prev = INFINITY;
  bool conv = false;
  double res[8];
  for (int sw = 0; sw < max_sweeps; ++sw) {
    {
      Timed tm(timer, KC_JAC_OTHER, s);
      if (!ok(launch_jacobi_sort_columns(jp, b.jb, s))) return out;
    }
    if (!ok(launch_jacobi_sweep(jp, b.jb, tol, s, timer))) return out;
    ++out.sweeps;
    if (!ok(hipMemcpyAsync(res, b.jb.result, sizeof(res), hipMemcpyDeviceToHost, s))) return out;
    if (!sync()) return out;
    const double off = res[3];
    if (trace >= 2) fprintf(stderr, "[ttm]   jacobi %dx%d sweep %d off=%.3e tol=%.3e\n", jp.L, jp.nc, sw, off, tol);
    if (!(off == off)) break;  // NaN
    if (off <= tol) {
      conv = true;
      break;
    }
    // Cyclic Jacobi converges quadratically at the end: after a sweep whose
    // largest scaled off-diagonal was off, what remains is of order off^2
    // (measured here: 3.6e-4 -> 7.9e-9 -> at the tolerance).  Once off^2 is
    // a hundredth of the tolerance the next sweep's rotations are below the
    // rounding level, so it is not run.
    if (off * off <= 0.01 * tol) {
      conv = true;
      break;
    }
    // stagnation at the rounding floor
    if (off < 1e3 * tol && off > 0.5 * prev) {
      conv = true;
      break;
    }
    prev = off;
  }
  if (!conv) {
    out.err = TTM_ENOCONV;
    set_last_error("one-sided Jacobi on the %d x %d factor of a %d x %d SVD did not converge in %d sweeps",
                   jp.L, jp.nc, p.np, p.no, out.sweeps);
    if (trace) fprintf(stderr, "[ttm] jacobi %dx%d did not converge\n", jp.L, jp.nc);
    return out;
  }
  // 4. singular values and the rank rule
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_jacobi_finish(jp, b.jb, eps, cap, forced, s, full_total))) return out;
  }
  if (!ok(hipMemcpyAsync(res, b.jb.result, sizeof(res), hipMemcpyDeviceToHost, s))) return out;
  if (!sync()) return out;
  if (res[4] != 0.0) {
    out.err = TTM_ENONFINITE;
    set_last_error("the singular values of a %d x %d SVD are not finite", p.np, p.no);
    return out;
  }
  out.rank = (int)res[0];
  out.disc = res[1];
  out.total = res[2];
  // 5. U_r = Q1 [U_W,r; 0] (no x r, column-major), then the caller's layout.
  // U_r^T row-major is that column-major matrix, so SVD_U_T is formed in u.
  const int r = out.rank;
  double *ucm = (u_layout == SVD_U_T) ? u : b.Xt;
  if (all) {
    // every resolved vector; U_r is their leading r columns
    const int kg = std::max(r, std::min(p.k, (int)res[6]));
    all->kg = kg;
    {
      Timed tm(timer, KC_JAC_OTHER, s);
      if (p.k < p.no && !ok(launch_fill(all->u, 0.0, (int64_t)p.no * kg, s))) return out;
      if (!ok(launch_jacobi_write_u(jp, b.jb, nullptr, kg, all->u, 1, p.no, s))) return out;
    }
    {
      Timed tm(timer, KC_QR, s);
      if (!ok(launch_apply_q(b.S, p.no, p.k, b.Tall, all->u, kg, b.qr, s))) return out;
    }
    {
      Timed tm(timer, KC_JAC_OTHER, s);
      if (!ok(launch_copy(ucm, all->u, (int64_t)p.no * r, s))) return out;
      hipLaunchKernelGGL(sorted_sigma_kernel, dim3((p.k + 255) / 256), dim3(256), 0, s, b.jb.sigma, b.jb.perm,
                         p.k, all->sigma);
      if (!ok(hipGetLastError())) return out;
    }
  } else {
    {
      Timed tm(timer, KC_JAC_OTHER, s);
      if (p.k < p.no && !ok(launch_fill(ucm, 0.0, (int64_t)p.no * r, s))) return out;
      if (!ok(launch_jacobi_write_u(jp, b.jb, nullptr, r, ucm, 1, p.no, s))) return out;
    }
    {
      Timed tm(timer, KC_QR, s);
      if (!ok(launch_apply_q(b.S, p.no, p.k, b.Tall, ucm, r, b.qr, s))) return out;
    }
  }
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (u_layout == SVD_U && !ok(launch_transpose(u, ucm, r, p.no, s))) return out;
    if (sigma_out) {
      hipLaunchKernelGGL(sorted_sigma_kernel, dim3((p.k + 255) / 256), dim3(256), 0, s, b.jb.sigma, b.jb.perm,
                         p.k, sigma_out);
      if (!ok(hipGetLastError())) return out;
    }
  }
  if (trace)
    fprintf(stderr, "[ttm] svd %dx%d sweeps=%d rank=%d disc=%.3e total=%.3e\n", p.np, p.no, out.sweeps,
            out.rank, out.disc, out.total);
  return out;
}

}  // namespace ttm
