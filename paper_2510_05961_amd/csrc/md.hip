// md.hip -- molecular dynamics around the MSM forward: charged
// Lennard-Jones particles (Sec. MD simulation of charged Lennard-Jonesium),
// integrated with velocity Verlet.  One step is a short launch sequence on
// the driver's stream (kick and drift, the MSM energy and forces through
// msm_energy_forces, the Lennard-Jones forces, kick and the step's energies);
// msm_md_run captures it once in a HIP graph and replays the graph.  With a
// Verlet skin on the plan (msm_plan_set_skin) the MSM cell list is rebuilt
// only when a charge has moved more than half the skin, decided on the
// device, so the same graph serves every step.
//
// Lennard-Jones part: u(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] S(r) with the
// quintic switch S = 1 - 10 x^3 + 15 x^4 - 6 x^5, x = (r - r_on)/(r_c - r_on)
// on r_on < r < r_c (S = 1 below, 0 above: u and its first two derivatives
// go to zero at r_c), over minimum images on periodic axes (r_c at most half
// a periodic edge).  All pairs, in LDS tiles of 256 particles: the driver is
// meant for the paper's N = 10^3 demonstration, not for large N.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "msm.h"
#include "plan_state.hpp"

using namespace msm;

struct msm_md_s {
  msm_plan plan = nullptr;
  int n = 0, fp64 = 0, cap = 0;
  double dt = 0, eps = 0, sigma = 0, rc = 0, ron = 0;
  double box[3] = {0, 0, 0};
  int per[3] = {0, 0, 0};
  hipStream_t s = nullptr;
  hipEvent_t ev[2] = {};
  // device state in the plan's precision: positions, velocities, total and
  // MSM forces [n][3]; charges, masses [n]
  void *pos = nullptr, *vel = nullptr, *F = nullptr, *Fc = nullptr, *q = nullptr, *m = nullptr;
  double* E = nullptr;    // [1] MSM energy of the last evaluation
  double* elj = nullptr;  // [1] its Lennard-Jones energy
  double* log = nullptr;  // [cap][3]: kinetic, Lennard-Jones and MSM energy after each step
  int* counter = nullptr; // steps logged since msm_md_set_state
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void*> allocs;
};

namespace {

template <typename T>
struct LJParams {
  T box[3];
  int per[3];
  T eps4, s2, rc2, ron, inv_w;  // 4 eps, sigma^2, r_c^2, r_on, 1/(r_c - r_on)
  T rc;
};

// v += dt/2 F/m, x += dt v; clears the Lennard-Jones energy of the step
template <typename T>
__global__ void k_md_kick_drift(int n, T* __restrict__ x, T* __restrict__ v,
                                const T* __restrict__ F, const T* __restrict__ m, T dt,
                                double* __restrict__ elj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *elj = 0.0;
  if (i >= 3 * n) return;
  const T vi = v[i] + T(0.5) * dt * F[i] / m[i / 3];
  v[i] = vi;
  x[i] += dt * vi;
}

// F = Fc + F_LJ over all pairs (LDS tiles of 256 j), E_LJ summed in FP64
template <typename T>
__global__ void __launch_bounds__(256)
    k_md_lj(int n, const T* __restrict__ x, LJParams<T> lp, const T* __restrict__ Fc,
            T* __restrict__ F, double* __restrict__ elj) {
  __shared__ T tile[256][3];
  __shared__ double part[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  T xi[3] = {T(0), T(0), T(0)};
  if (i < n)
    for (int k = 0; k < 3; ++k) xi[k] = x[3 * i + k];
  T f[3] = {T(0), T(0), T(0)};
  double e = 0.0;
  for (int j0 = 0; j0 < n; j0 += 256) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    for (int k = 0; k < 3; ++k) tile[threadIdx.x][k] = j < n ? x[3 * j + k] : T(0);
    __syncthreads();
    const int jn = min(256, n - j0);
    if (i < n) {
      for (int jj = 0; jj < jn; ++jj) {
        if (j0 + jj == i) continue;
        T d[3];
        for (int k = 0; k < 3; ++k) {
          d[k] = xi[k] - tile[jj][k];
          if (lp.per[k]) d[k] -= lp.box[k] * rint(d[k] / lp.box[k]);
        }
        const T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < lp.rc2)) continue;
        const T r = sqrt(r2);
        const T sr2 = lp.s2 / r2, sr6 = sr2 * sr2 * sr2;
        const T u = lp.eps4 * (sr6 * sr6 - sr6);
        const T du = lp.eps4 * (T(-12) * sr6 * sr6 + T(6) * sr6) / r;  // du/dr
        T S = T(1), dS = T(0);
        if (r > lp.ron) {
          const T t = (r - lp.ron) * lp.inv_w, t2 = t * t, t3 = t2 * t;
          S = T(1) - T(10) * t3 + T(15) * t3 * t - T(6) * t3 * t2;
          dS = (T(-30) * t2 + T(60) * t3 - T(30) * t3 * t) * lp.inv_w;
        }
        const T c = -(du * S + u * dS) / r;  // F_i = c d
        for (int k = 0; k < 3; ++k) f[k] += c * d[k];
        e += 0.5 * (double)(u * S);
      }
    }
  }
  if (i < n)
    for (int k = 0; k < 3; ++k) F[3 * i + k] = Fc[3 * i + k] + f[k];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) e += __shfl_xor(e, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(elj, part[0] + part[1] + part[2] + part[3]);
}

// v += dt/2 F/m; the step's kinetic energy (FP64) and its Lennard-Jones and
// MSM energies go to log[counter]
template <typename T>
__global__ void __launch_bounds__(256)
    k_md_kick(int n, T* __restrict__ v, const T* __restrict__ F, const T* __restrict__ m, T dt,
              const double* __restrict__ E, const double* __restrict__ elj,
              double* __restrict__ log, const int* __restrict__ counter, int cap) {
  __shared__ double part[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (i < n) {
    const T inv = T(1) / m[i];
    double v2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      const T vk = v[3 * i + k] + T(0.5) * dt * F[3 * i + k] * inv;
      v[3 * i + k] = vk;
      v2 += (double)vk * (double)vk;
    }
    ke = 0.5 * (double)m[i] * v2;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) ke += __shfl_xor(ke, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = ke;
  __syncthreads();
  const int c = *counter;
  if (threadIdx.x == 0 && c < cap) {
    atomicAdd(&log[3 * (size_t)c], part[0] + part[1] + part[2] + part[3]);
    if (blockIdx.x == 0) {
      log[3 * (size_t)c + 1] = *elj;
      log[3 * (size_t)c + 2] = *E;
    }
  }
}

__global__ void k_md_step_done(int* counter) {
  if (threadIdx.x == 0) *counter += 1;
}

template <typename T>
LJParams<T> lj_params(const msm_md_s* md) {
  LJParams<T> lp;
  for (int k = 0; k < 3; ++k) {
    lp.box[k] = (T)md->box[k];
    lp.per[k] = md->per[k];
  }
  lp.eps4 = (T)(4.0 * md->eps);
  lp.s2 = (T)(md->sigma * md->sigma);
  lp.rc2 = (T)(md->rc * md->rc);
  lp.rc = (T)md->rc;
  lp.ron = (T)md->ron;
  lp.inv_w = (T)(1.0 / (md->rc - md->ron));
  return lp;
}

// forces of the current positions: MSM through the library's own entry
// point, then the Lennard-Jones part added
template <typename T>
msm_status md_forces(msm_md md) {
  const msm_status st = msm_energy_forces(md->plan, md->n, md->pos, md->q, nullptr, md->E,
                                          md->Fc, nullptr, md->s);
  if (st != MSM_OK) return st;
  const int nb = (md->n + 255) / 256;
  hipLaunchKernelGGL(k_md_lj<T>, dim3(nb), dim3(256), 0, md->s, md->n, (const T*)md->pos,
                     lj_params<T>(md), (const T*)md->Fc, (T*)md->F, md->elj);
  return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

template <typename T>
msm_status md_step(msm_md md) {
  const int n = md->n;
  hipLaunchKernelGGL(k_md_kick_drift<T>, dim3((3 * n + 255) / 256), dim3(256), 0, md->s, n,
                     (T*)md->pos, (T*)md->vel, (const T*)md->F, (const T*)md->m, (T)md->dt,
                     md->elj);
  msm_status st = md_forces<T>(md);
  if (st != MSM_OK) return st;
  hipLaunchKernelGGL(k_md_kick<T>, dim3((n + 255) / 256), dim3(256), 0, md->s, n, (T*)md->vel,
                     (const T*)md->F, (const T*)md->m, (T)md->dt, (const double*)md->E,
                     (const double*)md->elj, md->log, (const int*)md->counter, md->cap);
  hipLaunchKernelGGL(k_md_step_done, dim3(1), dim3(64), 0, md->s, md->counter);
  return hipGetLastError() == hipSuccess ? MSM_OK : MSM_ERR_HIP;
}

msm_status md_alloc(msm_md md, void** p, size_t bytes) {
  if (hipMalloc(p, std::max(bytes, size_t(16))) != hipSuccess) {
    *p = nullptr;
    return MSM_ERR_OOM;
  }
  md->allocs.push_back(*p);
  return MSM_OK;
}

void md_free(msm_md md) {
  if (!md) return;
  (void)hipDeviceSynchronize();
  if (md->exec) (void)hipGraphExecDestroy(md->exec);
  if (md->graph) (void)hipGraphDestroy(md->graph);
  for (auto& e : md->ev)
    if (e) (void)hipEventDestroy(e);
  if (md->s) (void)hipStreamDestroy(md->s);
  for (void* p : md->allocs) (void)hipFree(p);
  delete md;
}

// the driver's stream follows the caller's, or the caller's the driver's
msm_status md_join(hipStream_t from, hipStream_t to, hipEvent_t e) {
  if (hipEventRecord(e, from) != hipSuccess || hipStreamWaitEvent(to, e, 0) != hipSuccess)
    return MSM_ERR_HIP;
  return MSM_OK;
}

}  // namespace

extern "C" {

msm_status msm_md_create(msm_md* out, msm_plan plan, int n, double dt, double lj_epsilon,
                         double lj_sigma, double lj_cutoff, double lj_switch_on, int log_steps) {
  if (!out) return MSM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!plan || plan->batch || n < 1 || log_steps < 0 || !(dt > 0) || !(lj_epsilon >= 0) ||
      !(lj_sigma > 0) || !(lj_switch_on >= 0) || !(lj_cutoff > lj_switch_on))
    return MSM_ERR_INVALID_ARG;
  if (!plan->device) return MSM_ERR_NO_DEVICE;
  if (plan->hp.tri) return MSM_ERR_UNSUPPORTED;
  if (n > plan->hp.max_n) return MSM_ERR_CAPACITY;
  for (int k = 0; k < 3; ++k)
    if (plan->hp.periodic[k] && lj_cutoff > 0.5 * plan->hp.box[k]) return MSM_ERR_CUTOFF_TOO_LARGE;
  msm_md md = new (std::nothrow) msm_md_s;
  if (!md) return MSM_ERR_OOM;
  md->plan = plan;
  md->n = n;
  md->fp64 = plan->hp.precision == MSM_FP64;
  md->cap = log_steps;
  md->dt = dt;
  md->eps = lj_epsilon;
  md->sigma = lj_sigma;
  md->rc = lj_cutoff;
  md->ron = lj_switch_on;
  for (int k = 0; k < 3; ++k) {
    md->box[k] = plan->hp.box[k];
    md->per[k] = plan->hp.periodic[k];
  }
  const size_t ts = md->fp64 ? sizeof(double) : sizeof(float);
  msm_status st = MSM_OK;
  if ((st = md_alloc(md, &md->pos, 3 * ts * n)) || (st = md_alloc(md, &md->vel, 3 * ts * n)) ||
      (st = md_alloc(md, &md->F, 3 * ts * n)) || (st = md_alloc(md, &md->Fc, 3 * ts * n)) ||
      (st = md_alloc(md, &md->q, ts * n)) || (st = md_alloc(md, &md->m, ts * n)) ||
      (st = md_alloc(md, (void**)&md->E, sizeof(double))) ||
      (st = md_alloc(md, (void**)&md->elj, sizeof(double))) ||
      (st = md_alloc(md, (void**)&md->log, 3 * sizeof(double) * (size_t)std::max(log_steps, 1))) ||
      (st = md_alloc(md, (void**)&md->counter, sizeof(int)))) {
    md_free(md);
    return st;
  }
  if (hipStreamCreateWithFlags(&md->s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&md->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&md->ev[1], hipEventDisableTiming) != hipSuccess) {
    md_free(md);
    return MSM_ERR_HIP;
  }
  *out = md;
  return MSM_OK;
}

msm_status msm_md_destroy(msm_md md) {
  md_free(md);
  return MSM_OK;
}

msm_status msm_md_set_state(msm_md md, const void* pos, const void* vel, const void* q,
                            const void* mass, void* stream) {
  if (!md || !pos || !vel || !q || !mass) return MSM_ERR_INVALID_ARG;
  const size_t ts = md->fp64 ? sizeof(double) : sizeof(float), n = (size_t)md->n;
  hipStream_t cs = (hipStream_t)stream;
  msm_status st;
  if ((st = md_join(cs, md->s, md->ev[0]))) return st;
  if (hipMemcpyAsync(md->pos, pos, 3 * ts * n, hipMemcpyDeviceToDevice, md->s) ||
      hipMemcpyAsync(md->vel, vel, 3 * ts * n, hipMemcpyDeviceToDevice, md->s) ||
      hipMemcpyAsync(md->q, q, ts * n, hipMemcpyDeviceToDevice, md->s) ||
      hipMemcpyAsync(md->m, mass, ts * n, hipMemcpyDeviceToDevice, md->s) ||
      hipMemsetAsync(md->log, 0, 3 * sizeof(double) * (size_t)std::max(md->cap, 1), md->s) ||
      hipMemsetAsync(md->counter, 0, sizeof(int), md->s) ||
      hipMemsetAsync(md->elj, 0, sizeof(double), md->s))
    return MSM_ERR_HIP;
  // the forces of the initial positions (an eager call: it also leaves the
  // plan's cell list and skin state ready for a captured step)
  st = md->fp64 ? md_forces<double>(md) : md_forces<float>(md);
  if (st != MSM_OK) return st;
  return md_join(md->s, cs, md->ev[1]);
}

msm_status msm_md_run(msm_md md, int nsteps, int use_graph, void* stream) {
  if (!md || nsteps < 0) return MSM_ERR_INVALID_ARG;
  hipStream_t cs = (hipStream_t)stream;
  msm_status st;
  if ((st = md_join(cs, md->s, md->ev[0]))) return st;
  if (use_graph && !md->exec && nsteps > 0) {
    if (hipStreamBeginCapture(md->s, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return MSM_ERR_HIP;
    st = md->fp64 ? md_step<double>(md) : md_step<float>(md);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(md->s, &g);
    if (st != MSM_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st != MSM_OK ? st : MSM_ERR_HIP;
    }
    md->graph = g;
    if (hipGraphInstantiate(&md->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      md->exec = nullptr;
      return MSM_ERR_HIP;
    }
  }
  for (int k = 0; k < nsteps; ++k) {
    if (use_graph) {
      if (hipGraphLaunch(md->exec, md->s) != hipSuccess) return MSM_ERR_HIP;
    } else if ((st = md->fp64 ? md_step<double>(md) : md_step<float>(md))) {
      return st;
    }
  }
  return md_join(md->s, cs, md->ev[1]);
}

msm_status msm_md_get_state(msm_md md, void* pos, void* vel, void* forces, void* stream) {
  if (!md) return MSM_ERR_INVALID_ARG;
  const size_t b = 3 * (md->fp64 ? sizeof(double) : sizeof(float)) * (size_t)md->n;
  hipStream_t cs = (hipStream_t)stream;
  msm_status st;
  if ((st = md_join(cs, md->s, md->ev[0]))) return st;
  if ((pos && hipMemcpyAsync(pos, md->pos, b, hipMemcpyDeviceToDevice, md->s)) ||
      (vel && hipMemcpyAsync(vel, md->vel, b, hipMemcpyDeviceToDevice, md->s)) ||
      (forces && hipMemcpyAsync(forces, md->F, b, hipMemcpyDeviceToDevice, md->s)))
    return MSM_ERR_HIP;
  return md_join(md->s, cs, md->ev[1]);
}

msm_status msm_md_energies(msm_md md, double* host, int max_steps, int* steps) {
  if (!md || !steps || max_steps < 0 || (max_steps > 0 && !host)) return MSM_ERR_INVALID_ARG;
  int c = 0;
  if (hipStreamSynchronize(md->s) != hipSuccess ||
      hipMemcpy(&c, md->counter, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    return MSM_ERR_HIP;
  *steps = c;
  const int k = std::min(std::min(c, md->cap), max_steps);
  if (k > 0 && hipMemcpy(host, md->log, 3 * sizeof(double) * (size_t)k, hipMemcpyDeviceToHost) !=
                   hipSuccess)
    return MSM_ERR_HIP;
  return MSM_OK;
}

}  // extern "C"
