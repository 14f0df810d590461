// Captured SR iterations and the numeric fault check.
//
// pvr_sr_graph_create records the library's own launches of `iters` SR
// iterations (simulate with residual, robust weights, gather adjoint, update;
// every problem of the plan in each launch) on a private capture stream and
// instantiates the graph; replays then issue the whole batch's work without
// host involvement.  Everything that needs the host (the adjoint's brick
// index, which sizes its lists with a readback) is prepared before the
// capture.  Kernel arguments are fixed at capture, so a graph is only valid
// for the plan state it was recorded from: every build, PSF or tile change
// and index rebuild bumps the plan's generation, and a launch against a
// newer generation is refused.
#include "pvr_internal.h"
#include "pvr_util.h"

#include <utility>

using namespace pvr;

struct pvr_sr_graph {
  pvr_plan *plan;
  long long generation;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" pvr_status pvr_check(pvr_plan *p, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!p) return fail(PVR_EINVAL, "pvr_check: plan is NULL");
  if (!p->attached) return PVR_OK;  // nothing has run
  unsigned flags = 0;
  HIP_TRY(hipMemcpyAsync(&flags, p->d_status, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (!flags) return PVR_OK;
  launch_fill_i32((int *)p->d_status, 0, 1, stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(stream));
  if (flags & PVR_FAULT_INDEX)
    return fail(PVR_ESHAPE, "pvr_check: the adjoint's index outgrew its capacity%s%s",
                (flags & PVR_FAULT_VOLUME) ? "; non-finite updated volume (pvr_sr_update)" : "",
                (flags & PVR_FAULT_RESIDUAL) ? "; non-finite residual statistics" : "");
  return fail(PVR_ENUMERIC, "pvr_check: non-finite values:%s%s",
              (flags & PVR_FAULT_VOLUME) ? " updated volume (pvr_sr_update)" : "",
              (flags & PVR_FAULT_RESIDUAL) ? " residual statistics (pvr_robust_weights)" : "");
  PVR_API_END();
}

extern "C" pvr_status pvr_sr_graph_create(pvr_plan *plan, float *X, float *X_alt,
                                          const float *y_obs, float *resid, float *p, float *pbar,
                                          float *patch_w, float *num, float *den,
                                          pvr_em_state *em, const pvr_sr_params *params,
                                          int32_t iters, hipStream_t stream,
                                          pvr_sr_graph **out) {
  PVR_API_BEGIN();
  PVR_ALIGNED("pvr_sr_graph_create", X, 4);
  PVR_ALIGNED("pvr_sr_graph_create", X_alt, 4);
  PVR_ALIGNED("pvr_sr_graph_create", y_obs, 4);
  PVR_ALIGNED("pvr_sr_graph_create", resid, 4);
  PVR_ALIGNED("pvr_sr_graph_create", p, 4);
  PVR_ALIGNED("pvr_sr_graph_create", pbar, 4);
  PVR_ALIGNED("pvr_sr_graph_create", patch_w, 4);
  PVR_ALIGNED("pvr_sr_graph_create", num, 4);
  PVR_ALIGNED("pvr_sr_graph_create", den, 4);
  PVR_ALIGNED("pvr_sr_graph_create", em, 8);
  if (!out) return fail(PVR_EINVAL, "pvr_sr_graph_create: out is NULL");
  *out = nullptr;
  if (!plan || !X || !X_alt || !y_obs || !resid || !p || !pbar || !patch_w || !num || !den ||
      !em || !params)
    return fail(PVR_EINVAL, "pvr_sr_graph_create: NULL argument");
  if (X == X_alt) return fail(PVR_EINVAL, "pvr_sr_graph_create: X and X_alt must differ");
  if (iters < 1) return fail(PVR_EINVAL, "pvr_sr_graph_create: iters must be >= 1");
  if (!plan->built) return fail(PVR_EINVAL, "pvr_sr_graph_create: build the plan first");
  if (plan->timing)
    return fail(PVR_EUNSUPPORTED, "pvr_sr_graph_create: switch kernel timing off before capturing");
  if (!plan->index_valid) {
    const pvr_status st = plan_build_index(plan, stream);
    if (st != PVR_OK) return st;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  hipStream_t cs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    HIP_TRY(e);
  }
  pvr_status st = PVR_OK;
  float *cur = X, *nxt = X_alt;
  for (int i = 0; i < iters && st == PVR_OK; ++i) {
    st = pvr_simulate(plan, cur, y_obs, nullptr, resid, cs);
    if (st == PVR_OK)
      st = pvr_robust_weights(plan, resid, y_obs, em, p, pbar, patch_w,
                              PVR_EM_RESID_FRESH | PVR_EM_PREP_ADJOINT, cs);
    if (st == PVR_OK) st = pvr_backproject(plan, resid, p, patch_w, num, den, cs);
    if (st == PVR_OK) st = pvr_sr_update(plan, cur, num, den, params, nxt, cs);
    std::swap(cur, nxt);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (st != PVR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;  // the failing call's message stands
  }
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    HIP_TRY(e);
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    HIP_TRY(e);
  }
  *out = new pvr_sr_graph{plan, plan->generation, g, x};
  return PVR_OK;
  PVR_API_END();
}

extern "C" pvr_status pvr_sr_graph_launch(const pvr_sr_graph *g, hipStream_t stream) {
  PVR_API_BEGIN();
  if (!g) return fail(PVR_EINVAL, "pvr_sr_graph_launch: graph is NULL");
  if (g->plan->generation != g->generation)
    return fail(PVR_EINVAL, "pvr_sr_graph_launch: the plan changed since the capture "
                            "(build, PSF, tiles or adjoint index); capture again");
  HIP_TRY(hipGraphLaunch(g->exec, stream));
  return PVR_OK;
  PVR_API_END();
}

extern "C" void pvr_sr_graph_destroy(pvr_sr_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}
