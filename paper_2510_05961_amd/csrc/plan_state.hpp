// plan_state.hpp -- the opaque msm_plan object shared by the C-ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "msm.h"
#include "plan.hpp"

namespace msm {
struct BatchState;  // batch.hip
void destroy_batch(BatchState* b);
// sticky device error bits: 1 domain, 2 non-finite, 4 malformed batch offsets
constexpr int kFlagOffsets = 4;
}  // namespace msm

namespace msm {
// Working memory of one forward or backward call, overwritten by every call:
// per level the grid charge and potential (plan precision) and the FP64
// convolution buffers (ug: the convolution's output or atomic target; ut:
// the x pass of omega' on factored levels); the cell list and cluster
// layout of the particles; the short-range outputs.  counts must be zero on
// entry to a call (the cluster layout leaves it so), and cpos / cv hold the
// null j-group (far-away zero charges, zero vectors) at index null_h.
struct WorkBufs {
  void* qg[kMaxLevels] = {};
  void* eg[kMaxLevels] = {};
  double* ug[kMaxLevels] = {};
  double* ut[kMaxLevels] = {};
  int* cell_of = nullptr;
  int* rank = nullptr;
  int* counts = nullptr;
  int* start = nullptr;
  int* perm = nullptr;
  // 8-particle clusters of the short-range sum: offsets per cell, padded
  // slots (x, y, z, q), boxes (lo, hi), info (first sorted index, count,
  // cell), force cotangent in slot order (backward)
  int* cl_start = nullptr;
  int* scan_tmp = nullptr;  // block totals of the many-workgroup cell scan
  void* cpos = nullptr;
  void* cbox = nullptr;
  int4* cinfo = nullptr;
  void* cv = nullptr;
  void* wrapped = nullptr;
  void* sorted = nullptr;
  void* phi0 = nullptr;
  void* F0 = nullptr;
  int null_h = 0;  // index of the null j-group in cpos / cv
};
}  // namespace msm

// Event-pair stage timer (enabled by msm_plan_set_profiling).
struct StageProfiler {
  bool on = false;
  std::vector<std::string> only;  // stages to record (empty: all)
  struct Pending {
    std::string stage;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<double, long>> total;
  // start and end of each stage after the first stage of its call ("bin" in
  // the forward, "bwd_layout" in the backward), summed like total
  std::map<std::string, std::pair<double, double>> offsets;
  hipEvent_t get() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  // returns an index to close with end(), or -1 when off
  int begin(const char* stage, hipStream_t s) {
    if (!on) return -1;
    if (!only.empty()) {
      bool want = false;
      for (const auto& o : only) want = want || o == stage;
      if (!want) return -1;
    }
    Pending p{stage, get(), get()};
    if (!p.a || !p.b) return -1;
    (void)hipEventRecord(p.a, s);
    pending.push_back(p);
    return (int)pending.size() - 1;
  }
  void end(int idx, hipStream_t s) {
    if (idx >= 0) (void)hipEventRecord(pending[idx].b, s);
  }
  void collect() {
    hipEvent_t anchor = nullptr;
    for (auto& p : pending) {
      float ms = 0.f;
      if (p.stage == "bin" || p.stage == "bwd_layout") anchor = p.a;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto& t = total[p.stage];
        t.first += ms;
        t.second += 1;
        float t0 = 0.f, t1 = 0.f;
        if (anchor && hipEventElapsedTime(&t0, anchor, p.a) == hipSuccess &&
            hipEventElapsedTime(&t1, anchor, p.b) == hipSuccess) {
          auto& o = offsets[p.stage];
          o.first += t0;
          o.second += t1;
        }
      }
    }
    for (auto& p : pending) {
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  ~StageProfiler() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct msm_plan_s {
  // batched plans (msm_batch_plan_create) keep their state here
  msm::BatchState* bs = nullptr;
  msm::HostPlan hp;
  StageProfiler prof;
  bool device = false;
  int device_id = -1;  // the GPU the plan's memory lives on
  bool batch = false;
  int ncell = 0;
  // device buffers (T = plan precision); stencils in FP64 with zero-padded
  // rows (conv_row_stride) and per-row non-zero x ranges
  double* K64[msm::kMaxLevels] = {};
  int2* rowext64[msm::kMaxLevels] = {};
  // geometry of the uploaded stencils (direct K, factored-level samples S)
  msm::ConvGeom kgeom[msm::kMaxLevels] = {}, sgeom[msm::kMaxLevels] = {};
  // factored levels: FP64 k-samples and their row extents
  double* S[msm::kMaxLevels] = {};
  int2* srowext[msm::kMaxLevels] = {};
  // working memory of the calls (own: allocated with the plan for max_n;
  // w points at the set the current call uses)
  msm::WorkBufs own;
  msm::WorkBufs* w = &own;
  void* Jd = nullptr;
  int* flag = nullptr;
  // Verlet skin (msm_plan_set_skin): device state [force, rebuild, calls,
  // rebuilds] (force: the next call rebuilds, after a new cell or skin or a
  // call that kept its cell list in a workspace), each charge's position and
  // wrap at the last rebuild (max_n vec4 each), and the n of the last call
  int* skin_state = nullptr;
  void* skin_ref = nullptr;
  void* skin_shift = nullptr;
  int skin_n = -1;
  // cells per axis the working memory was laid out for (later cell lists
  // never have more)
  int nc_cap[3] = {0, 0, 0};
  // cell derivative (msm_energy_forces_cell_gradient, triclinic plans): the
  // levels' derivative stencils T^l_ab and the top level's dK^L/dH_rc as
  // uploaded (built at the first such call after a cell change), and FP64
  // working grids plus the accumulators
  double* TS[msm::kMaxLevels][6] = {};
  int2* TSext[msm::kMaxLevels][6] = {};
  msm::ConvGeom tsgeom[msm::kMaxLevels][6] = {};
  double* dKd[9] = {};
  int2* dKext[9] = {};
  msm::ConvGeom dkgeom[9] = {};
  double* sgrid = nullptr;  // 3 FP64 grids of level 1's size, then 30 accumulators
  double* cellm = nullptr;  // H^{-1} (9 doubles, device)
  bool stress_ready = false;
  // side streams of the forward DAG (default priority, non-blocking) and the
  // fork/join events between them and the caller's stream
  hipStream_t sb = nullptr, sc = nullptr, sd = nullptr;
  hipEvent_t ev[6] = {};
  std::vector<void*> allocs;
};


namespace msm {
// device allocation owned by the plan (freed with it)
msm_status hip_alloc(msm_plan P, void** ptr, size_t bytes);
}  // namespace msm
std::string describe_batch(const msm::BatchState& B);
