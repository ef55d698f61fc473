// adamw.hip -- the first-order inner solver of a time step (Sec. 4.5, without
// constraint terms): the velocity v minimises the incremental potential whose
// gradient is g(v) = M (v - v_n)/h + f_int(q_n + h v, v) - f_ext, by AdamW, the
// Adam method with decoupled weight decay (Loshchilov and Hutter, ICLR 2019):
//   m <- b1 m + (1 - b1) g,   s <- b2 s + (1 - b2) g^2            (moments)
//   v <- v - lr (m / (1 - b1^l) / (sqrt(s / (1 - b2^l)) + eps) + wd v)
// at iteration l, then q = q_n + h v for the next force evaluation.
//
// Arranged for the GPU: each inner iteration is four launches on the caller's
// stream.  A one-lane kernel advances the iteration counter and forms the two
// bias-correction factors in device memory (so no per-DOF power is taken and
// the captured arguments never change); one per-DOF kernel applies the moment
// and velocity updates fused with q = q_n + h v; then the internal force (both
// passes of the force-only assembly) and the gradient over the mass rows.  The
// iterations between two convergence checks are captured once into a HIP graph
// and replayed.  Convergence (||g|| <= eps_in (1 + ||v||) or ||g|| <= eps_rel
// ||g_0||, g_0 the first gradient) is checked on the host from norms reduced on
// the device in a fixed order.
#include <cmath>

#include "tlfea_internal.h"

using tlfea::Mesh;

namespace tlfea {
namespace {

constexpr int kNormBlocks = 256;

struct AdamwArgs {
  double lr, beta1, beta2, eps, wd, h;
};

__global__ void k_fill(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// the iteration counter l and the bias-correction divisors 1 - b1^l, 1 - b2^l
__global__ void k_count(AdamwArgs p, int64_t* l, double* corr) {
  if (threadIdx.x != 0) return;
  const int64_t it = *l + 1;
  *l = it;
  corr[0] = 1.0 - std::pow(p.beta1, (double)it);
  corr[1] = 1.0 - std::pow(p.beta2, (double)it);
}

// per DOF: the two moments, the decoupled-decay velocity update and the step map
__global__ void k_adamw(AdamwArgs p, const double* __restrict__ corr, int64_t n, const double* __restrict__ g,
                        const double* __restrict__ q_n, double* __restrict__ m, double* __restrict__ s,
                        double* __restrict__ v, double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double gi = g[i];
  const double mi = p.beta1 * m[i] + (1.0 - p.beta1) * gi;
  const double si = p.beta2 * s[i] + (1.0 - p.beta2) * gi * gi;
  m[i] = mi;
  s[i] = si;
  const double vi = v[i];
  const double vn = vi - p.lr * ((mi / corr[0]) / (std::sqrt(si / corr[1]) + p.eps) + p.wd * vi);
  v[i] = vn;
  q[i] = q_n[i] + p.h * vn;
}

// partial sums of g.g and v.v per block (fixed order), then one block adds them
__global__ __launch_bounds__(256) void k_norms(const double* g, const double* v, int64_t n, double* part) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    a += g[i] * g[i];
    b += v[i] * v[i];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_norms_final(const double* part, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  out[0] = std::sqrt(a);
  out[1] = std::sqrt(b);
}

int blocks_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 1 << 20); }

}  // namespace
}  // namespace tlfea

namespace {

// one inner iteration on stream s (no allocation, no synchronisation)
int adamw_iteration(tlfea_mesh_t mesh, const tlfea::AdamwArgs& a, const double* q_n, const double* v_n,
                    const double* f_ext, double* v, double* q, double* m, double* sm, double* g, double* f,
                    int64_t* d_l, hipStream_t s) {
  const Mesh& me = mesh->m;
  const int64_t n = me.n_dof;
  double* corr = reinterpret_cast<double*>(d_l + 1);  // the two divisors follow the counter
  hipLaunchKernelGGL(tlfea::k_count, dim3(1), dim3(64), 0, s, a, d_l, corr);
  hipLaunchKernelGGL(tlfea::k_adamw, dim3(tlfea::blocks_for(n)), dim3(256), 0, s, a, corr, n, g, q_n, m, sm, v,
                     q);
  TLFEA_HIP_CHECK(hipGetLastError());
  int rc = tlfea_internal_force(mesh, q, v, f, s);
  if (rc) return rc;
  return tlfea_newton_gradient(mesh, v, v_n, f, f_ext, a.h, g, s);
}

}  // namespace

TLFEA_API int tlfea_adamw_solve(tlfea_mesh_t mesh, const tlfea_adamw_params* p, double h, const double* d_q_n,
                                const double* d_v_n, const double* d_f_ext, double* d_v, double* d_q,
                                double* d_work, int32_t max_iters, int32_t check_every, double eps_in,
                                double eps_rel, int32_t* iters_out, double* gnorm_out, void* stream) {
  if (!mesh || !p || !d_q_n || !d_v_n || !d_v || !d_q || !d_work || max_iters < 1 || check_every < 1 ||
      !(h > 0.0) || !std::isfinite(h) || !(p->lr > 0.0) || !(p->beta1 >= 0.0 && p->beta1 < 1.0) ||
      !(p->beta2 >= 0.0 && p->beta2 < 1.0) || !(p->eps > 0.0) || !(p->weight_decay >= 0.0) ||
      !(eps_in >= 0.0) || !(eps_rel >= 0.0))
    return TLFEA_ERR_INVALID;
  Mesh& m = mesh->m;
  if (!m.has_pattern) return TLFEA_ERR_NO_PATTERN;
  if (!m.d_mass) return TLFEA_ERR_INVALID;
  if (hipSetDevice(m.device) != hipSuccess) return TLFEA_ERR_HIP;
  auto s = (hipStream_t)stream;
  if (!s) return TLFEA_ERR_INVALID;  // the legacy stream cannot be captured
  const int64_t n = m.n_dof;
  double* mom = d_work;
  double* sec = d_work + n;
  double* g = d_work + 2 * n;
  double* f = d_work + 3 * n;
  // device scalars: iteration counter, bias-correction divisors, norm partials and norms
  if (!m.d_solver) {
    if (hipMalloc(&m.d_solver, sizeof(double) * (2 * tlfea::kNormBlocks + 6)) != hipSuccess) {
      (void)hipGetLastError();
      return TLFEA_ERR_NOMEM;
    }
  }
  auto* d_l = reinterpret_cast<int64_t*>(m.d_solver);
  double* part = m.d_solver + 3;
  double* norms = m.d_solver + 3 + 2 * tlfea::kNormBlocks;
  const tlfea::AdamwArgs a{p->lr, p->beta1, p->beta2, p->eps, p->weight_decay, h};
  // g = m = s = 0 and l = 0 (fill kernels: nothing here is a memset)
  hipLaunchKernelGGL(tlfea::k_fill, dim3(tlfea::blocks_for(3 * n)), dim3(256), 0, s, d_work, 3 * n);
  hipLaunchKernelGGL(tlfea::k_fill, dim3(1), dim3(64), 0, s, m.d_solver, (int64_t)1);
  TLFEA_HIP_CHECK(hipGetLastError());
  auto norms_to_host = [&](double* out) -> int {
    hipLaunchKernelGGL(tlfea::k_norms, dim3(tlfea::kNormBlocks), dim3(256), 0, s, g, d_v, n, part);
    hipLaunchKernelGGL(tlfea::k_norms_final, dim3(1), dim3(64), 0, s, part, tlfea::kNormBlocks, norms);
    TLFEA_HIP_CHECK(hipGetLastError());
    TLFEA_HIP_CHECK(hipMemcpyAsync(out, norms, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    TLFEA_HIP_CHECK(hipStreamSynchronize(s));
    return TLFEA_OK;
  };
  // the first iteration runs eagerly: it allocates what the assembly needs and gives g_0
  int rc = adamw_iteration(mesh, a, d_q_n, d_v_n, d_f_ext, d_v, d_q, mom, sec, g, f, d_l, s);
  if (rc) return rc;
  double nrm[2];
  if ((rc = norms_to_host(nrm))) return rc;
  const double g0 = nrm[0];
  int32_t done = 1;
  bool conv = nrm[0] <= eps_in * (1.0 + nrm[1]) || nrm[0] <= eps_rel * g0;
  hipGraphExec_t exec = nullptr;
  int32_t exec_len = 0;
  while (!conv && done < max_iters) {
    const int32_t chunk = std::min<int32_t>(check_every, max_iters - done);
    if (chunk != exec_len) {
      if (exec) (void)hipGraphExecDestroy(exec);
      exec = nullptr;
      TLFEA_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      for (int32_t i = 0; i < chunk && !rc; ++i)
        rc = adamw_iteration(mesh, a, d_q_n, d_v_n, d_f_ext, d_v, d_q, mom, sec, g, f, d_l, s);
      hipGraph_t graph = nullptr;
      const hipError_t e1 = hipStreamEndCapture(s, &graph);
      hipError_t e2 = hipSuccess;
      if (!rc && e1 == hipSuccess) e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (rc || e1 != hipSuccess || e2 != hipSuccess) {
        if (exec) (void)hipGraphExecDestroy(exec);
        (void)hipGetLastError();
        return rc ? rc : TLFEA_ERR_HIP;
      }
      exec_len = chunk;
    }
    if (hipGraphLaunch(exec, s) != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      return TLFEA_ERR_HIP;
    }
    done += chunk;
    if ((rc = norms_to_host(nrm))) {
      (void)hipGraphExecDestroy(exec);
      return rc;
    }
    conv = nrm[0] <= eps_in * (1.0 + nrm[1]) || nrm[0] <= eps_rel * g0;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (iters_out) *iters_out = done;
  if (gnorm_out) *gnorm_out = nrm[0];
  return TLFEA_OK;
}
