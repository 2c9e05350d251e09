// Adaptive multilevel Monte Carlo with parametric continuation (PC_MLMC,
// Section 5.1 Algorithm 1): the host loop that decides how many pairs each
// level needs (eq. MLMCSAMP) and hands every batch of pairs to the batched
// level estimator, which runs all the solves and the per-level sums on the
// device.  The host only combines a few double-double sums per level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rmg.h"
#include "rmg_host.hpp"

namespace {

int err(rmg_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return rmg::set_error(c, code, buf);
}

// Error-free transformation a + b = s + e (Knuth's TwoSum).
inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// a += b for double-double values hi + lo.
void dd_add(rmg_dd& a, const rmg_dd& b) {
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  e += a.lo + b.lo;
  two_sum(s, e, a.hi, a.lo);
}

inline double val(const rmg_dd& a) { return a.hi + a.lo; }

void accumulate(rmg_level_sums& acc, const rmg_level_sums& b) {
  acc.n += b.n;
  acc.n_failed += b.n_failed;
  acc.picard_its += b.picard_its;
  acc.mg_cycles += b.mg_cycles;
  acc.mg_cycles_coarse += b.mg_cycles_coarse;
  dd_add(acc.sY, b.sY);
  dd_add(acc.sY2, b.sY2);
  dd_add(acc.sQf, b.sQf);
  dd_add(acc.sQf2, b.sQf2);
  dd_add(acc.sQc, b.sQc);
  dd_add(acc.sQc2, b.sQc2);
}

// Sample variance from the sums of x and x^2 over n values (eq. MC_var).
double mc_var(int64_t n, const rmg_dd& s1, const rmg_dd& s2) {
  const double a = val(s1);
  return (val(s2) - a * a / (double)n) / (double)(n - 1);
}

// Bytes of device memory one solve on an n x n grid takes inside the level
// estimator (fields, head, previous water content, multigrid hierarchy), with
// room to spare; used only to size batches.
double solve_bytes(int n, int n_fields) {
  return (double)n * n * (8.0 * n_fields + 8.0 * 3 + 8.0 * 7 * 4.0 / 3.0) + 4096.0;
}

bool same_problem(const rmg_problem& a, const rmg_problem& b) {
  return a.model == b.model && a.n_steps == b.n_steps && a.qoi == b.qoi && a.theta_r == b.theta_r &&
         a.theta_s == b.theta_s && a.gardner_a == b.gardner_a && a.linear_c0 == b.linear_c0 &&
         a.vg_alpha_shift == b.vg_alpha_shift && a.vg_n_shift == b.vg_n_shift && a.h_top == b.h_top &&
         a.h_bottom == b.h_bottom && a.h_init == b.h_init && a.dt == b.dt && a.init_profile == b.init_profile &&
         a.init_rate == b.init_rate;
}

struct Staging {
  double* h = nullptr;
  double* d = nullptr;
  ~Staging() {
    if (h) (void)hipHostFree(h);
    if (d) (void)hipFree(d);
  }
};

}  // namespace

extern "C" {

int rmg_mlmc_optimal_samples(int n_levels, const double* V, const double* W, double eps, int64_t* N_out) {
  if (n_levels < 1 || n_levels > 16 || !V || !W || !N_out || !(eps > 0.0) || !std::isfinite(eps))
    return RMG_EINVAL;
  double tot = 0.0, c = 0.0;  // Neumaier sum of sqrt(V_k W_k)
  for (int l = 0; l < n_levels; ++l) {
    if (!(V[l] >= 0.0) || !(W[l] > 0.0) || !std::isfinite(V[l]) || !std::isfinite(W[l])) return RMG_EINVAL;
    const double t = std::sqrt(V[l] * W[l]);
    const double s = tot + t;
    c += std::fabs(tot) >= std::fabs(t) ? (tot - s) + t : (t - s) + tot;
    tot = s;
  }
  tot += c;
  for (int l = 0; l < n_levels; ++l) {
    const double N = std::ceil(tot * std::sqrt(V[l] / W[l]) / (eps * eps));
    if (!(N <= 4.6e18)) return RMG_EINVAL;
    N_out[l] = (int64_t)N;
  }
  return RMG_OK;
}

int pc_mlmc(rmg_ctx* ctx, int n_levels, const rmg_pc_level* L, int n_fields, int n_modes,
            const rmg_marginal* h_marg, const rmg_solver_opts* opts, const rmg_pc_opts* pc,
            rmg_xi_source xi, void* user, rmg_pc_level_out* out, rmg_pc_result* res, hipStream_t stream) {
  if (!ctx) return RMG_EINVAL;
  const auto t_start = std::chrono::steady_clock::now();
  if (n_levels < 1 || n_levels > 16 || !L || !h_marg || !opts || !pc || !xi || !out || !res)
    return err(ctx, RMG_EINVAL, "pc_mlmc: bad level count or NULL argument");
  if (n_fields < 1 || n_fields > 4 || n_modes < 1 || n_modes > 1024)
    return err(ctx, RMG_EINVAL, "pc_mlmc: bad n_fields / n_modes");
  if (!(pc->eps > 0.0) || !std::isfinite(pc->eps) || !(pc->bias_rate > 0.0) ||
      (pc->cost_model != RMG_COST_WORK && pc->cost_model != RMG_COST_TIME) || pc->max_rounds < 1 ||
      pc->max_rounds > 10000 || pc->max_pairs_per_call < 0 || pc->max_pairs_per_call > 32767)
    return err(ctx, RMG_EINVAL, "pc_mlmc: bad eps, bias_rate, cost_model, max_rounds or max_pairs_per_call");
  for (int l = 0; l < n_levels; ++l) {
    const rmg_pc_level& v = L[l];
    if (v.n_warmup < 2 || pc->max_pairs < v.n_warmup)
      return err(ctx, RMG_EINVAL, "pc_mlmc: level %d: n_warmup must be >= 2 and <= max_pairs", l);
    if (l == 0 ? v.n_coarse != 0 : (v.n_coarse != L[l - 1].n_fine || v.n_coarse * 2 != v.n_fine))
      return err(ctx, RMG_EINVAL, "pc_mlmc: level %d: n_coarse must be %s", l,
                 l == 0 ? "0" : "n_fine / 2 and the n_fine of the level below");
    if (l > 0 && !same_problem(v.coarse, L[l - 1].fine))
      return err(ctx, RMG_EINVAL, "pc_mlmc: level %d: coarse problem differs from level %d's fine problem", l,
                 l - 1);
  }

  // pairs per level per batched call
  std::vector<int64_t> cap(n_levels, pc->max_pairs_per_call);
  if (pc->max_pairs_per_call == 0) {
    size_t fr = 0, total = 0;
    if (hipSetDevice(rmg::device_of(ctx)) != hipSuccess || hipMemGetInfo(&fr, &total) != hipSuccess)
      return err(ctx, RMG_EHIP, "pc_mlmc: hipMemGetInfo failed");
    const double share = 0.5 * (double)fr / n_levels;
    for (int l = 0; l < n_levels; ++l) {
      const double b = solve_bytes(L[l].n_fine, n_fields) +
                       (L[l].n_coarse ? solve_bytes(L[l].n_coarse, n_fields) : 0.0) + 8.0 * n_fields * n_modes;
      cap[l] = std::max<int64_t>(1, std::min<int64_t>(32767, (int64_t)(share / b)));
    }
  }
  const size_t row = (size_t)n_fields * n_modes;
  std::vector<size_t> xoff(n_levels + 1, 0);
  for (int l = 0; l < n_levels; ++l) xoff[l + 1] = xoff[l] + (size_t)cap[l] * row;
  Staging st;
  if (hipSetDevice(rmg::device_of(ctx)) != hipSuccess ||
      hipHostMalloc((void**)&st.h, 8 * xoff[n_levels], hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&st.d, 8 * xoff[n_levels]) != hipSuccess)
    return err(ctx, RMG_ENOMEM, "pc_mlmc: cannot allocate the %zu-byte random-input staging buffers",
               8 * xoff[n_levels]);

  std::memset(out, 0, sizeof(rmg_pc_level_out) * n_levels);
  std::memset(res, 0, sizeof(rmg_pc_result));
  for (int l = 0; l < n_levels; ++l) out[l].target = L[l].n_warmup;

  // One batched call: every level in `which` draws up to its cap of the pairs it
  // still lacks; returns the call's wall milliseconds through *ms.
  auto batch = [&](const std::vector<int>& which, double* ms) -> int {
    std::vector<rmg_level> lv;
    std::vector<int> idx;
    for (int l : which) {
      const int64_t lack = out[l].target - out[l].sums.n;
      const int64_t room = pc->max_pairs - out[l].drawn;
      const int64_t cnt = std::min({lack, cap[l], room});
      if (cnt <= 0) continue;
      double* h = st.h + xoff[l];
      if (xi(user, l, out[l].drawn, cnt, h) != 0)
        return err(ctx, RMG_EINVAL, "pc_mlmc: the random-input source failed (level %d, pairs %lld..%lld)", l,
                   (long long)out[l].drawn, (long long)(out[l].drawn + cnt - 1));
      if (hipMemcpyAsync(st.d + xoff[l], h, 8 * cnt * row, hipMemcpyHostToDevice, stream) != hipSuccess)
        return err(ctx, RMG_EHIP, "pc_mlmc: random-input copy failed");
      rmg_level e{};
      e.n_fine = L[l].n_fine;
      e.n_coarse = L[l].n_coarse;
      e.n_samples = cnt;
      e.fine = L[l].fine;
      e.coarse = l ? L[l].coarse : L[l].fine;
      e.d_basis_fine = L[l].d_basis_fine;
      e.d_basis_coarse = L[l].d_basis_coarse;
      e.d_xi = st.d + xoff[l];
      lv.push_back(e);
      idx.push_back(l);
    }
    if (lv.empty()) return RMG_OK;
    std::vector<rmg_level_sums> s(lv.size());
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = mlmc_level_estimate(ctx, (int)lv.size(), lv.data(), n_fields, n_modes, h_marg, opts, s.data(),
                                       nullptr, stream);
    if (ms) *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rc != RMG_OK && rc != RMG_ENOTCONV) return rc;  // failed pairs are expected and excluded
    ++res->calls;
    for (size_t k = 0; k < idx.size(); ++k) {
      accumulate(out[idx[k]].sums, s[k]);
      out[idx[k]].drawn += lv[k].n_samples;
    }
    return RMG_OK;
  };
  // Draw until every level in `which` has `target` successful pairs or has
  // drawn max_pairs; accumulates the wall time per level in ms_acc if given.
  auto fill = [&](const std::vector<int>& which, std::vector<double>* ms_acc) -> int {
    for (;;) {
      std::vector<int> open;
      for (int l : which)
        if (out[l].sums.n < out[l].target && out[l].drawn < pc->max_pairs) open.push_back(l);
      if (open.empty()) return RMG_OK;
      double ms = 0.0;
      if (int rc = batch(open, &ms)) return rc;
      if (ms_acc)
        for (int l : open) (*ms_acc)[l] += ms;
    }
  };

  // Algorithm 1, steps 1-2: warm-up pairs N*_l on every level.  With the time
  // cost model each level runs alone, so its wall time is its own.
  std::vector<double> warm_ms(n_levels, 0.0);
  std::vector<int> all(n_levels);
  for (int l = 0; l < n_levels; ++l) all[l] = l;
  if (pc->cost_model == RMG_COST_TIME) {
    for (int l = 0; l < n_levels; ++l)
      if (int rc = fill({l}, &warm_ms)) return rc;
  } else if (int rc = fill(all, nullptr)) {
    return rc;
  }
  for (int l = 0; l < n_levels; ++l) {
    const rmg_level_sums& s = out[l].sums;
    if (s.n < 2)
      return err(ctx, RMG_ENOTCONV, "pc_mlmc: level %d: %lld successful warm-up pairs of %lld drawn (need 2)", l,
                 (long long)s.n, (long long)out[l].drawn);
    const double nf2 = (double)L[l].n_fine * L[l].n_fine, nc2 = (double)L[l].n_coarse * L[l].n_coarse;
    out[l].W = pc->cost_model == RMG_COST_TIME
                   ? warm_ms[l] / (double)out[l].drawn
                   : ((double)(s.mg_cycles - s.mg_cycles_coarse) * nf2 + (double)s.mg_cycles_coarse * nc2) /
                         (double)out[l].drawn;
    if (!(out[l].W > 0.0)) out[l].W = 1e-300;  // a level whose solves cost nothing measurable
  }

  // Steps 3-5: update N_l from eq. MLMCSAMP, draw what is missing, repeat.
  bool converged = false, exhausted = false;
  std::vector<double> V(n_levels), Wl(n_levels);
  std::vector<int64_t> N(n_levels);
  while (res->rounds < pc->max_rounds) {
    for (int l = 0; l < n_levels; ++l) {
      V[l] = std::max(0.0, mc_var(out[l].sums.n, out[l].sums.sY, out[l].sums.sY2));
      Wl[l] = out[l].W;
    }
    if (rmg_mlmc_optimal_samples(n_levels, V.data(), Wl.data(), pc->eps, N.data()) != RMG_OK)
      return err(ctx, RMG_EINVAL, "pc_mlmc: eq. MLMCSAMP gave no finite sample count");
    ++res->rounds;
    bool more = false;
    for (int l = 0; l < n_levels; ++l) {
      out[l].target = std::max<int64_t>(N[l], 2);
      more |= out[l].sums.n < out[l].target;
    }
    if (!more) {
      converged = true;
      break;
    }
    if (exhausted) break;
    if (int rc = fill(all, nullptr)) return rc;
    for (int l = 0; l < n_levels; ++l)
      exhausted |= out[l].sums.n < out[l].target && out[l].drawn >= pc->max_pairs;
  }

  // Results: eqs. MLMCestimator, ML_var, MLMCVar, discErr.
  rmg_dd mean{0.0, 0.0}, var{0.0, 0.0};
  double err2 = 0.0, cost = 0.0;
  for (int l = 0; l < n_levels; ++l) {
    rmg_pc_level_out& o = out[l];
    const rmg_level_sums& s = o.sums;
    o.V = std::max(0.0, mc_var(s.n, s.sY, s.sY2));
    o.mean = val(s.sY) / (double)s.n;
    dd_add(mean, rmg_dd{o.mean, 0.0});
    double vl = mc_var(s.n, s.sQf, s.sQf2);
    if (l > 0) vl -= mc_var(s.n, s.sQc, s.sQc2);
    dd_add(var, rmg_dd{vl, 0.0});
    err2 += o.V / (double)s.n;
    cost += (double)o.drawn * o.W;
  }
  res->mean = val(mean);
  res->var = val(var);
  res->sampling_err2 = err2;
  // Bias (eq. discErr with s = 2): the finest grid against the next coarser one under the
  // same parameter set Theta_L (eq. numErr fixes Theta_L).  With continuation the finest
  // level's coarse member solves Theta_{L-1}, so further pairs of the finest level (their
  // numbers continue the level's) are solved with Theta_L on both grids, as many as the
  // level's N_L (at least 2); without it the level's own pairs serve.
  res->bias = NAN;
  if (n_levels > 1) {
    const int lt = n_levels - 1;
    rmg_level_sums bs{};
    if (std::memcmp(&L[lt].coarse, &L[lt].fine, sizeof(rmg_problem)) == 0) {
      bs = out[lt].sums;
    } else {
      const int64_t want = std::max<int64_t>(2, out[lt].target);
      while (bs.n < want && out[lt].drawn + res->bias_pairs < pc->max_pairs) {
        const int64_t first = out[lt].drawn + res->bias_pairs;
        const int64_t cnt = std::min({want - bs.n, cap[lt], pc->max_pairs - first});
        double* h = st.h + xoff[lt];
        if (xi(user, lt, first, cnt, h) != 0)
          return err(ctx, RMG_EINVAL, "pc_mlmc: the random-input source failed (level %d, pairs %lld..%lld)", lt,
                     (long long)first, (long long)(first + cnt - 1));
        if (hipMemcpyAsync(st.d + xoff[lt], h, 8 * cnt * row, hipMemcpyHostToDevice, stream) != hipSuccess)
          return err(ctx, RMG_EHIP, "pc_mlmc: random-input copy failed");
        rmg_level e{};
        e.n_fine = L[lt].n_fine;
        e.n_coarse = L[lt].n_coarse;
        e.n_samples = cnt;
        e.fine = L[lt].fine;
        e.coarse = L[lt].fine;
        e.d_basis_fine = L[lt].d_basis_fine;
        e.d_basis_coarse = L[lt].d_basis_coarse;
        e.d_xi = st.d + xoff[lt];
        rmg_level_sums sb{};
        const int rc = mlmc_level_estimate(ctx, 1, &e, n_fields, n_modes, h_marg, opts, &sb, nullptr, stream);
        if (rc != RMG_OK && rc != RMG_ENOTCONV) return rc;
        ++res->calls;
        accumulate(bs, sb);
        res->bias_pairs += cnt;
        cost += (double)cnt * out[lt].W;
      }
    }
    if (bs.n > 0) res->bias = std::sqrt(val(bs.sY2) / (double)bs.n) / (std::pow(2.0, pc->bias_rate) - 1.0);
  }
  res->total_cost = cost;
  res->converged = converged && err2 <= pc->eps * pc->eps * (1.0 + 1e-12);
  res->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (!res->converged)
    return err(ctx, RMG_ENOTCONV, "pc_mlmc: stopped after %d N_l updates without reaching eps (%s)", res->rounds,
               exhausted ? "max_pairs reached" : "max_rounds reached");
  rmg::set_error(ctx, RMG_OK, "");
  return RMG_OK;
}

}  // extern "C"
