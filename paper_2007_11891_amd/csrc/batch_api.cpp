// Host side of the batched solver (include/hdg.h, "Batched solves"): one
// single-problem context per problem supplies the mesh records, the 1D
// tables, the Jacobi diagonal and the right-hand-side / recovery kernels; the
// batch owns the concatenated CG vectors, the work-unit schedule of the
// persistent kernel and the captured graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cmath>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/hdg.h"
#include "batch.hpp"
#include "hdg_internal.hpp"
#include "host_util.hpp"

using namespace hdg;

struct hdg_batch {
  int count = 0;
  double tau = 0.0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int device = 0;
  std::vector<hdg_ctx*> sub;
  std::vector<int64_t> off, voff;   // free-trace and volume offsets
  int64_t total_free = 0, total_vol = 0;
  int variant[kMaxNP + 1];          // tile variant per degree p (index p)
  std::vector<double> tabs;         // per-degree tables, packed as batch_tab_off
  double* d_tabs = nullptr;
  // concatenated FP64 vectors (total_free each)
  double* d_b = nullptr;
  double* d_x = nullptr;
  double* d_z = nullptr;
  double* d_p0 = nullptr;
  double* d_p1 = nullptr;
  double* d_qa = nullptr;
  double* d_qb = nullptr;
  double* d_dinv = nullptr;
  // one-phase form (see BatchArgs): second slots and its partials
  int form = 0;
  double* d_z1 = nullptr;
  double* d_s0 = nullptr;
  double* d_s1 = nullptr;
  double* d_qa1 = nullptr;
  double* d_qb1 = nullptr;
  double* d_pcg = nullptr;          // [2 * 3 * max_segs]
  // schedule
  int nblocks = 0;                  // persistent grid of the current form
  int n_cu = 0;                     // compute units of the device
  int nblocks_form[3] = {0, 0, 0};  // co-resident grid of each form
  int max_segs = 0;                 // bound on segments per phase: count + largest grid + 1
  std::vector<BatchProbDev> probs;
  BatchProbDev* d_probs = nullptr;
  MeshDev* d_meshes = nullptr;      // per-problem mesh records (pencil form)
  BatchSeg* d_useg = nullptr;       // [max_segs]
  BatchSeg* d_vseg = nullptr;       // [max_segs]
  int* d_useg_range = nullptr;      // [nblocks + 1]
  int* d_vseg_range = nullptr;      // [nblocks + 1]
  double* d_ppq = nullptr;          // [max_segs]
  double* d_prz = nullptr;          // [max_segs]
  double* d_prr = nullptr;
  unsigned* d_flags = nullptr;      // [2 * nblocks * kFlagStride]
  BatchState* d_A = nullptr;
  BatchState* d_B = nullptr;
  GridBar* d_bar = nullptr;
  BatchState* h_A = nullptr;        // pinned copies read after a solve
  GridBar* h_bar = nullptr;
  // probs array state on the device
  double probs_rtol2 = -1.0;
  int probs_maxit = -1;
  // captured pipeline
  hipGraphExec_t graph_pre = nullptr;    // full pipeline, or RHS + reset (split)
  hipGraphExec_t graph_post = nullptr;   // recovery (split mode only)
  bool split = false;
  const double* g_f = nullptr;
  double* g_trace = nullptr;
  double* g_uvol = nullptr;
  int g_max_iters = -1;
};

namespace {

// Relative cost of one apply work item, from per-segment timings of the
// persistent kernel at three blocks per CU on the 256-problem batch (p = 2..10):
// an element work unit keeps its block busy for nearly the same time in the
// two-phase form whatever its degree (the unit is bound by the latency of its
// dependent loads, not by its bytes; 12 % more from n_p = 8 on), and 11-13 us
// in the one-phase form; an element of a pencil column row takes 5-7 us.  A
// segment adds about two units' worth in the two-phase form (its partial
// sums and decisions): kSegCost, charged at the first unit of each problem.
constexpr double kSegCost = 14.0;
double item_cost(int form, int np) {
  switch (form) {
    case 1: return 10.2 + 0.25 * np;
    case 2: return 4.6 + 0.22 * np;
    default: return np >= 8 ? 7.85 : 7.0;
  }
}

// Share of a phase's work for the s-th block on a compute unit in the
// two-phase form (its blocks run in launch order, and the co-resident launch
// places blocks k, k + n_cu, ... on one CU).  The SIMDs issue from older
// waves first, so that the first block on a CU outruns the later ones: with
// equal shares at three blocks per CU, per-block timers of the 256-problem
// batch gave 4.1, 6.1 and 7.6 us per element work unit for the three slots,
// and each CU ran its last block alone for the last quarter of the apply
// phase.  At the two blocks per CU the form now runs, apply shares 1 : 0.70
// measured fastest (1 : 0.78 evens the mean end times of the two slots but
// measured 0.4 % slower: the phase ends with its slowest block, and blocks of
// one slot spread more than the slots differ); the streaming vector phase is
// barely uneven.  (The pencil form measured slower with unequal shares and
// the one-phase form remaps its blocks: both keep equal shares.)
double slot_share(int form, bool apply, int slot) {
  static const double wa[3] = {1.0, 0.70, 0.55};
  static const double wv[3] = {1.0, 0.98, 0.97};
  if (form != 0 || slot < 0) return 1.0;
  return (apply ? wa : wv)[slot < 3 ? slot : 2];
}

// Splits the problems' work into per-block segments.  Apply phase: the
// global list of work units (problem-major) is cut into nb contiguous ranges
// of about equal time (cost times the block's share), each range into one
// segment per problem it touches.  Vector phases: the concatenated free
// trace is cut into nb ranges in the same shares (multiples of 64 entries),
// likewise; a problem without free entries gets one empty segment.  Segments
// are listed block by block, so a problem's segments are consecutive in both
// lists.
hdg_status build_schedule(hdg_batch* b) {
  const int nb = b->nblocks;
  // cumulative shares: block k's part of the apply (vector) phase is
  // [wcum[k], wcum[k + 1]) ([vcum[k], vcum[k + 1]))
  std::vector<double> wcum(nb + 1, 0.0), vcum(nb + 1, 0.0);
  for (int k = 0; k < nb; ++k) {
    const int slot = b->n_cu > 0 ? k / b->n_cu : -1;
    wcum[k + 1] = wcum[k] + slot_share(b->form, true, slot);
    vcum[k + 1] = vcum[k] + slot_share(b->form, false, slot);
  }
  for (int k = 0; k <= nb; ++k) {
    wcum[k] /= wcum[nb];
    vcum[k] /= vcum[nb];
  }
  // apply work items of each problem: element work units (forms 0, 1) or
  // whole columns along x3 of EPB slots (pencil form), with their cost
  std::vector<int64_t> ubeg(b->count + 1, 0);
  std::vector<double> ucost(b->count, 0.0);
  for (int i = 0; i < b->count; ++i) {
    const hdg_ctx* c = b->sub[i];
    BatchProbDev& P = b->probs[i];
    P.variant = b->variant[c->p];
    const int epb = tile_epb(c->np, P.variant);
    if (b->form == 2) {
      ubeg[i + 1] = ubeg[i] + (int64_t)((c->n[0] + epb - 1) / epb) * c->n[1];
      ucost[i] = c->n[2] * item_cost(2, c->np);
    } else {
      ubeg[i + 1] = ubeg[i] + (c->n_elem + epb - 1) / epb;
      ucost[i] = item_cost(b->form, c->np);
    }
  }
  // apply segments: item u goes to the block holding the midpoint of its
  // cost interval; ucut[k] is the first item of block k
  const int64_t U = ubeg[b->count];
  std::vector<int64_t> ucut(nb + 1, U);
  {
    double total = 0.0;
    const double seg = b->form == 0 ? kSegCost : 0.0;
    for (int i = 0; i < b->count; ++i)
      total += (double)(ubeg[i + 1] - ubeg[i]) * ucost[i] + (ubeg[i + 1] > ubeg[i] ? seg : 0.0);
    if (!(total > 0.0)) total = 1.0;
    double acc = 0.0;
    int blk = 0, next = 1;
    ucut[0] = 0;
    for (int i = 0; i < b->count; ++i) {
      for (int64_t u = ubeg[i]; u < ubeg[i + 1]; ++u) {
        const double w = ucost[i] + (u == ubeg[i] ? seg : 0.0);
        const double mid = (acc + 0.5 * w) / total;
        while (blk + 1 < nb && wcum[blk + 1] <= mid) ++blk;
        while (next <= blk) ucut[next++] = u;
        acc += w;
      }
    }
  }
  std::vector<BatchSeg> useg, vseg;
  std::vector<int> urange(nb + 1), vrange(nb + 1);
  for (auto& P : b->probs) P.n_usegs = P.n_vsegs = 0;
  int prob = 0;
  for (int blk = 0; blk < nb; ++blk) {
    urange[blk] = (int)useg.size();
    for (int64_t u = ucut[blk]; u < ucut[blk + 1];) {
      while (ubeg[prob + 1] <= u) ++prob;
      const int64_t e = std::min(ucut[blk + 1], ubeg[prob + 1]);
      BatchProbDev& P = b->probs[prob];
      if (P.n_usegs++ == 0) P.useg_begin = (int)useg.size();
      useg.push_back(BatchSeg{prob, (int)(u - ubeg[prob]), (int)(e - ubeg[prob]), 0});
      u = e;
    }
  }
  urange[nb] = (int)useg.size();
  // vector segments: cut points on the concatenated free trace
  const int64_t N = b->total_free;
  std::vector<int64_t> vcut(nb + 1);
  for (int k = 0; k <= nb; ++k)
    vcut[k] = std::min<int64_t>(N, ((int64_t)std::llround((double)N * vcum[k]) + 32) / 64 * 64);
  vcut[0] = 0;
  vcut[nb] = N;
  int blk = 0;
  for (int i = 0; i < b->count; ++i) {
    BatchProbDev& P = b->probs[i];
    const int64_t lo0 = b->off[i], hi0 = b->off[i] + b->sub[i]->n_free;
    int64_t lo = lo0;
    do {
      // block whose range holds lo (an empty problem at the very end goes to the last block)
      while (blk + 1 < nb && vcut[blk + 1] <= lo) ++blk;
      const int64_t hi = std::min(hi0, vcut[blk + 1]);
      if (P.n_vsegs++ == 0) P.vseg_begin = (int)vseg.size();
      vseg.push_back(BatchSeg{i, (int)(lo - lo0), (int)(hi - lo0), blk});
      lo = hi;
    } while (lo < hi0);
  }
  // per-block ranges (the pad field held the block while building)
  {
    size_t k = 0;
    for (int bl = 0; bl <= nb; ++bl) {
      while (k < vseg.size() && vseg[k].pad < bl) ++k;
      vrange[bl] = (int)k;
    }
    vrange[nb] = (int)vseg.size();
    for (auto& sg : vseg) sg.pad = 0;
  }
  if ((int)useg.size() > b->max_segs || (int)vseg.size() > b->max_segs)
    return fail(HDG_EINVAL, "internal: schedule exceeds its buffers");
  for (const auto& P : b->probs)
    if (P.n_usegs < 1 || P.n_vsegs < 1) return fail(HDG_EINVAL, "internal: problem without segments");
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipMemcpy(b->d_useg, useg.data(), sizeof(BatchSeg) * useg.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_vseg, vseg.data(), sizeof(BatchSeg) * vseg.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_useg_range, urange.data(), sizeof(int) * urange.size(),
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_vseg_range, vrange.data(), sizeof(int) * vrange.size(),
                    hipMemcpyHostToDevice));
  b->probs_maxit = -1;   // force a re-upload of the problem records
  return HDG_OK;
}

hdg_status upload_probs(hdg_batch* b, double rtol2, int maxit) {
  if (b->probs_rtol2 == rtol2 && b->probs_maxit == maxit) return HDG_OK;
  for (auto& P : b->probs) {
    P.rtol2 = rtol2;
    P.maxit = maxit;
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipMemcpy(b->d_probs, b->probs.data(), sizeof(BatchProbDev) * b->probs.size(),
                    hipMemcpyHostToDevice));
  b->probs_rtol2 = rtol2;
  b->probs_maxit = maxit;
  return HDG_OK;
}

// max_iters: passes of the two-phase form for the solve asked; the one-phase
// form decides on iterate k - 1 in pass k and needs one pass more.
BatchArgs make_args(const hdg_batch* b, int max_iters) {
  BatchArgs a{};
  a.probs = b->d_probs;
  a.n_probs = b->count;
  a.max_iters = max_iters + (b->form == 1 ? 1 : 0);
  a.form = b->form;
  a.max_segs = b->max_segs;
  a.z1 = b->d_z1;
  a.s0 = b->d_s0;
  a.s1 = b->d_s1;
  a.qa1 = b->d_qa1;
  a.qb1 = b->d_qb1;
  a.pcg = b->d_pcg;
  a.useg = b->d_useg;
  a.useg_range = b->d_useg_range;
  a.vseg = b->d_vseg;
  a.vseg_range = b->d_vseg_range;
  a.x = b->d_x;
  a.z = b->d_z;
  a.p0 = b->d_p0;
  a.p1 = b->d_p1;
  a.qa = b->d_qa;
  a.qb = b->d_qb;
  a.dinv = b->d_dinv;
  a.b = b->d_b;
  a.ppq = b->d_ppq;
  a.prz = b->d_prz;
  a.prr = b->d_prr;
  a.A = b->d_A;
  a.B = b->d_B;
  a.bar = b->d_bar;
  a.flags = b->d_flags;
  a.tabs = b->d_tabs;
  a.meshes = b->d_meshes;
  return a;
}

void drop_graphs(hdg_batch* b) {
  if (b->graph_pre) (void)hipGraphExecDestroy(b->graph_pre);
  if (b->graph_post) (void)hipGraphExecDestroy(b->graph_post);
  b->graph_pre = b->graph_post = nullptr;
  b->g_max_iters = -1;
}

// Right-hand sides of every problem (eigen basis) into d_b.
hipError_t enqueue_rhs(hdg_batch* b, const double* f, hipStream_t s) {
  for (int i = 0; i < b->count; ++i) {
    const hdg_ctx* c = b->sub[i];
    if (c->n_free == 0) continue;
    double* qa = b->d_qa + b->off[i];
    double* qb = b->d_qb + b->off[i];
    hipError_t e = launch_volume(c, VOL_RHS, 1, f + b->voff[i], nullptr, nullptr, nullptr, nullptr,
                                 qa, qb, nullptr, nullptr, s);
    if (e == hipSuccess) e = launch_combine<double>(qa, qb, b->d_b + b->off[i], c->n_free, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Nodal trace and (optionally) volume solution of every problem from d_x.
hipError_t enqueue_recovery(hdg_batch* b, const double* f, double* trace, double* u_vol,
                            hipStream_t s) {
  for (int i = 0; i < b->count; ++i) {
    const hdg_ctx* c = b->sub[i];
    const double* xh = c->n_free ? b->d_x + b->off[i] : nullptr;
    hipError_t e = hipSuccess;
    if (u_vol)
      e = launch_volume(c, VOL_RECON, 1, f + b->voff[i], xh, nullptr, nullptr, nullptr, nullptr,
                        nullptr, u_vol + b->voff[i], nullptr, s);
    if (e == hipSuccess && c->n_free)
      e = launch_face_transform<double>(c->np, c->d_mats64 + 2 * c->np * c->np, xh, nullptr,
                                        trace + b->off[i], c->n_free_faces, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hdg_status capture_end(hdg_batch* b, hipError_t launch_err, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
  if (launch_err != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return fail(HDG_EHIP, "graph capture failed: %s",
                hipGetErrorString(launch_err != hipSuccess ? launch_err : e2));
  }
  hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(HDG_EHIP, "graph instantiation failed: %s", hipGetErrorString(e3));
  }
  return HDG_OK;
}

// Capture the pipeline: [RHS, reset, persistent CG, recovery] in one graph,
// or, when the cooperative launch cannot be captured, [RHS, reset] and
// [recovery] with the CG launched directly between them.
hdg_status build_pipeline(hdg_batch* b, const double* f, double* trace, double* u_vol,
                          int max_iters) {
  if ((b->graph_pre || b->split) && b->g_f == f && b->g_trace == trace && b->g_uvol == u_vol &&
      b->g_max_iters == max_iters && b->graph_pre)
    return HDG_OK;
  drop_graphs(b);
  const BatchArgs args = make_args(b, max_iters);
  if (!b->split) {
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_rhs(b, f, b->cap_stream);
    if (e == hipSuccess) e = launch_batch_reset(b->d_A, b->d_B, b->d_bar, b->d_flags, b->count, b->nblocks, b->cap_stream);
    if (e == hipSuccess) e = launch_batch_cg(args, b->nblocks, b->cap_stream);
    if (e == hipSuccess) e = enqueue_recovery(b, f, trace, u_vol, b->cap_stream);
    if (capture_end(b, e, &b->graph_pre) != HDG_OK) b->split = true;
  }
  if (b->split) {
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_rhs(b, f, b->cap_stream);
    if (e == hipSuccess) e = launch_batch_reset(b->d_A, b->d_B, b->d_bar, b->d_flags, b->count, b->nblocks, b->cap_stream);
    ST_TRY(capture_end(b, e, &b->graph_pre));
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    e = enqueue_recovery(b, f, trace, u_vol, b->cap_stream);
    ST_TRY(capture_end(b, e, &b->graph_post));
  }
  b->g_f = f;
  b->g_trace = trace;
  b->g_uvol = u_vol;
  b->g_max_iters = max_iters;
  return HDG_OK;
}

hdg_status check_barrier(hdg_batch* b) {
  HIP_TRY(hipMemcpyAsync(b->h_bar, b->d_bar, sizeof(GridBar), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (b->h_bar->err)
    return fail(HDG_EHIP, "persistent CG: grid barrier timed out (blocks not co-resident)");
  return HDG_OK;
}

}  // namespace

extern "C" {

hdg_status hdg_batch_destroy(hdg_batch* b) {
  if (!b) return HDG_OK;
  if (b->stream || b->cap_stream) (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  for (hdg_ctx* c : b->sub) hdg_destroy(c);
  for (double** p : {&b->d_b, &b->d_x, &b->d_z, &b->d_p0, &b->d_p1, &b->d_qa, &b->d_qb,
                     &b->d_dinv, &b->d_ppq, &b->d_prz, &b->d_prr, &b->d_z1, &b->d_s0, &b->d_s1,
                     &b->d_qa1, &b->d_qb1, &b->d_pcg})
    dfree(*p);
  dfree(b->d_probs);
  dfree(b->d_meshes);
  dfree(b->d_useg);
  dfree(b->d_vseg);
  dfree(b->d_useg_range);
  dfree(b->d_vseg_range);
  dfree(b->d_flags);
  dfree(b->d_tabs);
  dfree(b->d_A);
  dfree(b->d_B);
  dfree(b->d_bar);
  if (b->h_A) (void)hipHostFree(b->h_A);
  if (b->h_bar) (void)hipHostFree(b->h_bar);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return HDG_OK;
}

hdg_status hdg_batch_create(int count, const int* n_elem3, const int* p, const double* lambda,
                            double tau_hat, void* stream, hdg_batch** out) {
  if (!out) return fail(HDG_EINVAL, "out is NULL");
  *out = nullptr;
  ST_TRY(validate_batch_create(count, n_elem3, p, lambda, tau_hat));
  hdg_batch* b = new (std::nothrow) hdg_batch();
  if (!b) return fail(HDG_ENOMEM, "host allocation failed");
  auto cleanup = [&](hdg_status st) {
    hdg_batch_destroy(b);
    return st;
  };
  b->count = count;
  b->tau = tau_hat;
  b->stream = reinterpret_cast<hipStream_t>(stream);
  for (int& v : b->variant) v = 0;
  if (hipGetDevice(&b->device) != hipSuccess) return cleanup(fail(HDG_EHIP, "no HIP device"));
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(fail(HDG_EHIP, "stream creation failed"));
  b->sub.assign(count, nullptr);
  b->off.assign(count, 0);
  b->voff.assign(count, 0);
  hdg_status st;
  for (int i = 0; i < count; ++i) {
    const int* ne = n_elem3 + 3 * i;
    std::vector<double> h[3];
    for (int a = 0; a < 3; ++a) h[a].assign(ne[a], 1.0 / ne[a]);
    if ((st = hdg_create(ne, h[0].data(), h[1].data(), h[2].data(), p[i], tau_hat, nullptr,
                         lambda[i], stream, &b->sub[i])) != HDG_OK)
      return cleanup(st);
    // the element pass addresses a problem's trace vectors with 32-bit byte
    // offsets below 2^31
    if (b->sub[i]->n_free >= ((int64_t)1 << 28) || b->sub[i]->n_elem > INT32_MAX)
      return cleanup(fail(HDG_EINVAL, "problem %d too large for the batched solver "
                                      "(free trace of 2^28 values or more)", i));
    b->off[i] = b->total_free;
    b->voff[i] = b->total_vol;
    b->total_free += b->sub[i]->n_free;
    b->total_vol += b->sub[i]->n_vol;
  }
  if (b->total_free > ((int64_t)1 << 40)) return cleanup(fail(HDG_EINVAL, "batch too large"));
  for (double** ptr : {&b->d_b, &b->d_x, &b->d_z, &b->d_p0, &b->d_p1, &b->d_qa, &b->d_qb,
                       &b->d_dinv, &b->d_z1, &b->d_s0, &b->d_s1, &b->d_qa1, &b->d_qb1})
    if ((st = dalloc(ptr, b->total_free)) != HDG_OK) return cleanup(st);
  // Jacobi inverse diagonals of the single-problem contexts
  for (int i = 0; i < count; ++i) {
    const hdg_ctx* c = b->sub[i];
    if (c->n_free && hipMemcpyAsync(b->d_dinv + b->off[i], c->d_tmp[3], sizeof(double) * c->n_free,
                                    hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
      return cleanup(fail(HDG_EHIP, "diagonal copy failed"));
  }
  // persistent grid of each form: every block resident (cooperative launch)
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
    return cleanup(fail(HDG_EHIP, "device attribute query failed"));
  int nb_max = 0;
  for (int form = 0; form < 3; ++form) {
    int per_cu = 0;
    if (batch_occupancy(form, &per_cu) != hipSuccess || per_cu < 1)
      return cleanup(fail(HDG_EHIP, "occupancy query of the persistent kernel failed"));
    b->nblocks_form[form] = std::min(per_cu, 4) * n_cu;
    nb_max = std::max(nb_max, b->nblocks_form[form]);
  }
  b->nblocks = b->nblocks_form[0];
  b->n_cu = n_cu;
  // each block range splits into at most one more segment than problems it touches
  b->max_segs = count + nb_max + 1;
  const int ms = b->max_segs;
  if ((st = dalloc(&b->d_probs, count)) != HDG_OK || (st = dalloc(&b->d_useg, ms)) != HDG_OK ||
      (st = dalloc(&b->d_vseg, ms)) != HDG_OK ||
      (st = dalloc(&b->d_useg_range, nb_max + 1)) != HDG_OK ||
      (st = dalloc(&b->d_vseg_range, nb_max + 1)) != HDG_OK ||
      (st = dalloc(&b->d_ppq, ms)) != HDG_OK || (st = dalloc(&b->d_prz, ms)) != HDG_OK ||
      (st = dalloc(&b->d_prr, ms)) != HDG_OK || (st = dalloc(&b->d_pcg, 6 * ms)) != HDG_OK ||
      (st = dalloc(&b->d_A, count)) != HDG_OK ||
      (st = dalloc(&b->d_B, count)) != HDG_OK || (st = dalloc(&b->d_bar, 1)) != HDG_OK ||
      (st = dalloc(&b->d_flags, 2 * (int64_t)nb_max * kFlagStride)) != HDG_OK)
    return cleanup(st);
  if (hipHostMalloc(reinterpret_cast<void**>(&b->h_A), sizeof(BatchState) * count,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->h_bar), sizeof(GridBar), hipHostMallocDefault) !=
          hipSuccess)
    return cleanup(fail(HDG_ENOMEM, "pinned host allocation failed"));
  b->probs.resize(count);
  b->tabs.assign(kBatchTabWords, 0.0);
  for (int i = 0; i < count; ++i) {
    const hdg_ctx* c = b->sub[i];
    BatchProbDev& P = b->probs[i];
    P = BatchProbDev{};
    P.info = c->d_info;
    P.lam = c->d_lam;
    P.n_elem = (int)c->n_elem;
    P.nff = (int)c->n_free_faces;
    P.np = c->np;
    P.off = b->off[i];
    P.n = c->n_free;
    // the free faces normal to x3 (all interior: batched problems are
    // Dirichlet on every side), as a DOF range of the problem's trace
    const int64_t npf = (int64_t)c->np * c->np;
    P.x3_lo = (int)(c->mesh.foff[2] * npf);
    P.x3_hi = (int)((c->mesh.foff[2] + (int64_t)c->n[0] * c->n[1] * (c->n[2] - 1)) * npf);
    // per-degree tables (one tau_hat for the whole batch)
    const int o = batch_tab_off(c->np);
    for (int k = 0; k < c->np; ++k) {
      b->tabs[o + k] = c->et64.bs0[k];
      b->tabs[o + c->np + k] = c->et64.bs1[k];
      b->tabs[o + 2 * c->np + k] = c->et64.lam[k];
    }
    b->tabs[o + 3 * c->np] = c->et64.H;
  }
  {
    std::vector<MeshDev> meshes(count);
    for (int i = 0; i < count; ++i) meshes[i] = b->sub[i]->mesh;
    if ((st = dalloc(&b->d_meshes, count)) != HDG_OK) return cleanup(st);
    if (hipMemcpy(b->d_meshes, meshes.data(), sizeof(MeshDev) * count, hipMemcpyHostToDevice) !=
        hipSuccess)
      return cleanup(fail(HDG_EHIP, "mesh record upload failed"));
  }
  if ((st = dalloc(&b->d_tabs, kBatchTabWords)) != HDG_OK) return cleanup(st);
  if (hipMemcpy(b->d_tabs, b->tabs.data(), sizeof(double) * kBatchTabWords,
                hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(HDG_EHIP, "table upload failed"));
  if ((st = build_schedule(b)) != HDG_OK) return cleanup(st);
  if (hipStreamSynchronize(b->stream) != hipSuccess)
    return cleanup(fail(HDG_EHIP, "batch setup failed: %s", hipGetErrorString(hipGetLastError())));
  *out = b;
  return HDG_OK;
}

hdg_status hdg_batch_sizes(const hdg_batch* b, int64_t* n_free, int64_t* n_vol,
                           int64_t* total_free, int64_t* total_vol) {
  if (!b) return fail(HDG_EINVAL, "batch is NULL");
  for (int i = 0; i < b->count; ++i) {
    if (n_free) n_free[i] = b->sub[i]->n_free;
    if (n_vol) n_vol[i] = b->sub[i]->n_vol;
  }
  if (total_free) *total_free = b->total_free;
  if (total_vol) *total_vol = b->total_vol;
  return HDG_OK;
}

hdg_status hdg_batch_set_tile(hdg_batch* b, int p, int variant) {
  if (!b) return fail(HDG_EINVAL, "batch is NULL");
  if (p < 0 || p > 10) return fail(HDG_EINVAL, "degree %d out of [0, 10]", p);
  if (variant < 0 || variant >= kNumTileVariants)
    return fail(HDG_EINVAL, "tile variant must be in [0, %d)", kNumTileVariants);
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (p == 0) {
    for (int& v : b->variant) v = variant;
  } else {
    b->variant[p] = variant;
  }
  drop_graphs(b);
  return build_schedule(b);
}

hdg_status hdg_batch_set_form(hdg_batch* b, int form) {
  if (!b) return fail(HDG_EINVAL, "batch is NULL");
  if (form < 0 || form > 2) return fail(HDG_EINVAL, "form must be 0, 1 or 2, got %d", form);
  HIP_TRY(hipStreamSynchronize(b->stream));
  // every form has its own grid, work item and item cost: a new schedule
  b->form = form;
  b->nblocks = b->nblocks_form[form];
  drop_graphs(b);
  return build_schedule(b);
}

hdg_status hdg_batch_form(const hdg_batch* b, int* form) {
  if (!b || !form) return fail(HDG_EINVAL, "NULL argument");
  *form = b->form;
  return HDG_OK;
}

hdg_status hdg_batch_tiles(const hdg_batch* b, int* variants) {
  if (!b || !variants) return fail(HDG_EINVAL, "NULL argument");
  for (int q = 0; q <= kMaxNP - 1; ++q) variants[q] = -1;
  for (const hdg_ctx* c : b->sub) variants[c->p] = b->variant[c->p];
  return HDG_OK;
}

hdg_status hdg_batch_time_cg(hdg_batch* b, int iters, int reps, double* ms) {
  if (!b || !ms || iters < 1 || reps < 1) return fail(HDG_EINVAL, "invalid argument");
  ST_TRY(upload_probs(b, 0.0, iters));   // never converges, stops at the cap
  HIP_TRY(launch_fill64(b->d_b, 1.0, b->total_free, b->stream));
  const BatchArgs args = make_args(b, iters + 1);
  HIP_TRY(launch_batch_reset(b->d_A, b->d_B, b->d_bar, b->d_flags, b->count, b->nblocks, b->stream));
  HIP_TRY(launch_batch_cg(args, b->nblocks, b->stream));   // warm-up
  ST_TRY(check_barrier(b));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float total = 0.f;
  hipError_t err = hipSuccess;
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    err = launch_batch_reset(b->d_A, b->d_B, b->d_bar, b->d_flags, b->count, b->nblocks, b->stream);
    if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
    if (err == hipSuccess) err = launch_batch_cg(args, b->nblocks, b->stream);
    if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    total += t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(err);
  ST_TRY(check_barrier(b));
  *ms = (double)total / reps;
  return HDG_OK;
}

hdg_status hdg_batch_autotune(hdg_batch* b, int iters, int reps, int* variants) {
  if (!b || iters < 1 || reps < 1) return fail(HDG_EINVAL, "invalid argument");
  // degrees by decreasing share of the work (elements x n_p^3)
  double work[kMaxNP + 1] = {0};
  for (const hdg_ctx* c : b->sub) work[c->p] += (double)c->n_elem * c->np * c->np * c->np;
  std::vector<int> degs;
  for (int q = 1; q <= 10; ++q)
    if (work[q] > 0.0) degs.push_back(q);
  std::sort(degs.begin(), degs.end(), [&](int x, int y) { return work[x] > work[y]; });
  auto measure = [&](double* best) -> hdg_status {
    double m = 1e300;
    for (int r = 0; r < reps; ++r) {
      double t = 0.0;
      ST_TRY(hdg_batch_time_cg(b, iters, 1, &t));
      m = std::min(m, t);
    }
    *best = m;
    return HDG_OK;
  };
  // each form with its own tile search; the faster (form, tiles) pair stays
  double best_all = 1e300;
  int best_form = 0;
  int best_var[kMaxNP + 1];
  for (int form = 0; form <= 2; ++form) {
    ST_TRY(hdg_batch_set_form(b, form));
    ST_TRY(hdg_batch_set_tile(b, 0, 0));
    double best = 0.0;
    ST_TRY(measure(&best));
    for (int q : degs) {
      int keep = b->variant[q];
      for (int v = 1; v < kNumTileVariants; ++v) {
        ST_TRY(hdg_batch_set_tile(b, q, v));
        double t = 0.0;
        ST_TRY(measure(&t));
        if (t < best) {
          best = t;
          keep = v;
        }
      }
      ST_TRY(hdg_batch_set_tile(b, q, keep));
    }
    if (best < best_all) {
      best_all = best;
      best_form = form;
      std::copy(b->variant, b->variant + kMaxNP + 1, best_var);
    }
  }
  ST_TRY(hdg_batch_set_form(b, best_form));
  for (int q : degs) ST_TRY(hdg_batch_set_tile(b, q, best_var[q]));
  if (variants) ST_TRY(hdg_batch_tiles(b, variants));
  return HDG_OK;
}

hdg_status hdg_batch_solve_forcing(hdg_batch* b, const double* f, double* trace_free,
                                   double* u_vol, const hdg_solve_opts* opts,
                                   hdg_batch_result* results, double* t_ms) {
  if (!b || !f || !trace_free) return fail(HDG_EINVAL, "NULL argument");
  hdg_solve_opts o;
  hdg_default_opts(&o);
  if (opts) o = *opts;
  if (!(o.rtol > 0.0) || o.maxit < 1 || o.check_every < 1 || o.precond < 0 || o.precond > 3)
    return fail(HDG_EINVAL, "invalid solver options");
  if (o.precond != 1)
    return fail(HDG_EUNSUPPORTED, "the batched solver runs the transformed (precond 1) CG only");
  if (o.mixed) return fail(HDG_EUNSUPPORTED, "the batched solver runs in FP64 only");
  ST_TRY(upload_probs(b, o.rtol * o.rtol, o.maxit));
  // the apply that detects the stop also applies the last x update: one more pass
  ST_TRY(build_pipeline(b, f, trace_free, u_vol, o.maxit + 1));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  hipError_t err = hipEventRecord(e0, b->stream);
  if (err == hipSuccess) err = hipGraphLaunch(b->graph_pre, b->stream);
  if (b->split) {
    if (err == hipSuccess) err = launch_batch_cg(make_args(b, o.maxit + 1), b->nblocks, b->stream);
    if (err == hipSuccess) err = hipGraphLaunch(b->graph_post, b->stream);
  }
  if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(b->h_A, b->d_A, sizeof(BatchState) * b->count, hipMemcpyDeviceToHost,
                         b->stream);
  if (err == hipSuccess)
    err = hipMemcpyAsync(b->h_bar, b->d_bar, sizeof(GridBar), hipMemcpyDeviceToHost, b->stream);
  if (err == hipSuccess) err = hipStreamSynchronize(b->stream);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(err);
  if (t_ms) *t_ms = t;
  if (b->h_bar->err)
    return fail(HDG_EHIP, "persistent CG: grid barrier timed out (blocks not co-resident)");
  hdg_status overall = HDG_OK;
  int bad = -1;
  for (int i = 0; i < b->count; ++i) {
    const BatchState& s = b->h_A[i];
    hdg_batch_result r{};
    r.iters = s.iter;
    r.status = s.done == 1 ? HDG_OK : (s.done == 2 ? HDG_ENOCONV : HDG_EHIP);
    const double rr0 = s.rr_stop / (o.rtol * o.rtol);
    r.rel_res = rr0 > 0.0 ? std::sqrt(s.rr / rr0) : 0.0;
    if (s.done == 0) r.status = HDG_EHIP;   // never finished: should not happen
    if (r.status != HDG_OK && bad < 0) bad = i;
    if (results) results[i] = r;
  }
  if (bad >= 0) {
    const int d = b->h_A[bad].done;
    overall = d == 2 ? HDG_ENOCONV : HDG_EHIP;
    fail(overall, "problem %d stopped after %d iterations (%s)", bad, b->h_A[bad].iter,
         d == 2 ? "iteration cap" : (d == 3 ? "CG breakdown" : "not finished"));
  }
  return overall;
}

}  // extern "C"
