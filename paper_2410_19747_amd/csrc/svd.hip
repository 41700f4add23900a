// Truncated SVD driver for the swap and rounding steps: column ordering,
// Householder QR preconditioning, one-sided Jacobi on R^T, rank rule and
// write-out (the steps are listed with svd_oside in ttm_internal.h).
#include <math.h>
#include <stdio.h>

#include <algorithm>

#include "ttm_internal.h"

namespace ttm {
namespace {
constexpr double kUnitRoundoff = 2.220446049250313e-16;

size_t r32(size_t n) { return (n + 31) & ~(size_t)31; }

struct SvdBufs {
  double *S = nullptr;      // np x no: ordered copy of Y, factored in place
  double *qr = nullptr;     // QR scratch
  double *ynorm = nullptr;  // no column norms of Y
  int *perm0 = nullptr;     // no: ordered position -> column of Y
  JacobiBufs jb;
};

SvdBufs carve(const SvdPlan &p, double *base) {
  SvdBufs b;
  double *q = base;
  auto adv = [&](size_t nd) {
    double *x = q;
    q += r32(nd);
    return x;
  };
  const JacobiPlan &jp = p.jp;
  b.S = adv((size_t)p.np * p.no);
  b.qr = adv(qr_inplace_scratch_doubles(p.np, p.no));
  b.ynorm = adv((size_t)p.no);
  b.perm0 = reinterpret_cast<int *>(adv((size_t)p.no));
  b.jb.W = adv((size_t)jp.L * jp.ncp);
  b.jb.Wt = adv((size_t)jp.L * jp.ncp);
  b.jb.part = adv((size_t)jp.pairs * jp.sw * 4 * jp.bw * jp.bw);
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

SvdPlan svd_plan(int np, int no) {
  SvdPlan p;
  p.np = np;
  p.no = no;
  p.k = std::min(np, no);
  p.jp = jacobi_plan(no, p.k);
  return p;
}

size_t svd_ws_doubles(const SvdPlan &p) {
  const JacobiPlan &jp = p.jp;
  size_t n = 0;
  n += r32((size_t)p.np * p.no);
  n += r32(qr_inplace_scratch_doubles(p.np, p.no));
  n += 2 * r32((size_t)p.no);
  n += 2 * r32((size_t)jp.L * jp.ncp);
  n += r32((size_t)jp.pairs * jp.sw * 4 * jp.bw * jp.bw);
  n += r32((size_t)jp.rounds * jp.pairs);
  n += r32((size_t)jp.pairs * 4 * jp.bw * jp.bw);
  n += r32((size_t)jp.pairs);
  n += 2 * r32((size_t)jp.ncp);
  n += r32(8);
  return n;
}

SvdResult svd_oside(const SvdPlan &p, const double *Y, double eps, int cap, int forced, int max_sweeps,
                    double *u, int u_layout, double *sigma_out, double *ws, hipStream_t s,
                    KernelTimer *timer, int trace) {
  SvdResult out;
  SvdBufs b = carve(p, ws);
  const JacobiPlan &jp = p.jp;
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess) {
      out.err = TTM_EHIP;
      if (trace) fprintf(stderr, "[ttm] HIP error %s\n", hipGetErrorString(e));
      return false;
    }
    return true;
  };
  auto sync = [&]() {
    if (!ok(hipStreamSynchronize(s))) return false;
    if (timer && timer->on) timer->collect();
    return true;
  };
  // 1-2. column order, copy, ||Y||_F^2, QR
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_column_norms(Y, p.np, p.no, b.ynorm, s))) return out;
    if (!ok(launch_sort_desc(b.ynorm, p.no, b.perm0, s))) return out;
    if (!ok(launch_gather_columns(Y, b.perm0, p.np, p.no, b.S, s))) return out;
    if (!ok(launch_frob_from_norms(b.ynorm, p.no, b.jb.result, s))) return out;
  }
  {
    Timed tm(timer, KC_QR, s);
    // Block column pivoting in the QR saves Jacobi sweeps (the rows of R come
    // out graded); its selection step pays off once a sweep is expensive.
    int *pivot = (p.no >= 2048) ? b.perm0 : nullptr;
    if (!ok(launch_qr_inplace(b.S, p.np, p.no, b.qr, pivot, s))) return out;
  }
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_rt_from_qr(b.S, p.np, p.no, p.k, jp.ncp, b.jb.W, s))) return out;
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
    // stagnation at the rounding floor
    if (off < 1e3 * tol && off > 0.5 * prev) {
      conv = true;
      break;
    }
    prev = off;
  }
  if (!conv) {
    out.err = TTM_ENOCONV;
    if (trace) fprintf(stderr, "[ttm] jacobi %dx%d did not converge\n", jp.L, jp.nc);
    return out;
  }
  // 4. singular values and the rank rule
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_jacobi_finish(jp, b.jb, eps, cap, forced, s))) return out;
  }
  if (!ok(hipMemcpyAsync(res, b.jb.result, sizeof(res), hipMemcpyDeviceToHost, s))) return out;
  if (!sync()) return out;
  if (res[4] != 0.0) {
    out.err = TTM_ENONFINITE;
    return out;
  }
  out.rank = (int)res[0];
  out.disc = res[1];
  out.total = res[2];
  // 5. U_r in the caller's layout
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    const int64_t u_os = (u_layout == SVD_U) ? out.rank : 1;
    const int64_t u_ts = (u_layout == SVD_U) ? 1 : p.no;
    if (!ok(launch_jacobi_write_u(jp, b.jb, b.perm0, out.rank, u, u_os, u_ts, s))) return out;
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
