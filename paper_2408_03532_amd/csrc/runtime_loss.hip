// C ABI of the amplitude loss and its gradient.
#include <string>

#include "internal.hpp"
#include "loss.hpp"

namespace pftpie {
namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace: spectra u_j (when the backward recomputes them), per-wave loss
// partials, back-projected residuals R_j [J][n][n] for the gradient gathers.
struct LossLayout {
  size_t U, part, R, Pp, total;
};

LossLayout loss_layout(const pie_scan_s* s) {
  LossLayout L;
  L.U = 0;
  L.part = al256((size_t)s->J * s->plan->m * s->plan->m * 8);
  L.R = L.part + al256((size_t)s->J * 4 * 8);
  L.Pp = L.R + al256((size_t)s->J * s->plan->n * s->plan->n * 8);
  L.total = L.Pp + al256((size_t)((s->J + 63) / 64) * s->plan->n * s->plan->n * 8);
  return L;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

pftpie_status check_common(const pie_scan_s* s, const void* O, const void* P, const float* amp, void* ws,
                           size_t ws_bytes, const char* who) {
  if (!s) return fail(PFTPIE_E_INVALID, std::string(who) + ": scan is NULL");
  if (!O || !P || !amp) return fail(PFTPIE_E_INVALID, std::string(who) + ": NULL object, probe or amplitudes");
  if ((uintptr_t)O % 8 || (uintptr_t)P % 8 || (uintptr_t)amp % 4)
    return fail(PFTPIE_E_INVALID, std::string(who) + ": misaligned object, probe or amplitudes");
  const LossLayout L = loss_layout(s);
  if (!ws || ws_bytes < L.total)
    return fail(PFTPIE_E_INVALID, std::string(who) + ": workspace smaller than amp_loss_workspace_size (" +
                                      std::to_string(L.total) + " bytes)");
  if ((uintptr_t)ws % 256) return fail(PFTPIE_E_INVALID, std::string(who) + ": workspace must be 256-byte aligned");
  return PFTPIE_OK;
}

LossArgs base_args(const pie_scan_s* s, const void* O, const void* P, const float* amp, void* ws) {
  const pftpie_plan_s* pl = s->plan;
  const LossLayout L = loss_layout(s);
  LossArgs a{};
  a.n = pl->n;
  a.m = pl->m;
  a.nb = pl->nb;
  a.mt = pl->mt;
  a.J = s->J;
  a.H = s->H;
  a.W = s->W;
  a.pos = s->pos;
  a.fa = pl->fa;
  a.ft = pl->ft;
  a.fa_bytes = pl->fa_bytes;
  a.ft_bytes = pl->ft_bytes;
  a.num_cu = pl->num_cu;
  a.prec = pl->prec;
  a.O = static_cast<const float2*>(O);
  a.P = static_cast<const float2*>(P);
  a.amp = amp;
  a.part = reinterpret_cast<double*>(static_cast<char*>(ws) + L.part);
  a.Rbuf = reinterpret_cast<float2*>(static_cast<char*>(ws) + L.R);
  a.gPpart = reinterpret_cast<float2*>(static_cast<char*>(ws) + L.Pp);
  a.bb_r0 = s->bb_r0;
  a.bb_c0 = s->bb_c0;
  a.bb_h = s->bb_h;
  a.bb_w = s->bb_w;
  a.tiles_x = s->tiles_x;
  a.tiles_y = s->tiles_y;
  a.tile_ptr = s->tile_ptr;
  a.tile_pos = s->tile_pos;
  return a;
}

}  // namespace
}  // namespace pftpie

using namespace pftpie;

extern "C" {

pftpie_status amp_loss_workspace_size(pie_scan scan, size_t* bytes) {
  if (!scan || !bytes) return fail(PFTPIE_E_INVALID, "amp_loss_workspace_size: NULL argument");
  *bytes = loss_layout(scan).total;
  return PFTPIE_OK;
}

pftpie_status amp_loss_forward(pie_scan scan, const void* object, const void* probe, const float* amp,
                               double* loss_dev, void* saved_u, void* workspace, size_t ws_bytes, void* stream) {
  if (pftpie_status st = check_common(scan, object, probe, amp, workspace, ws_bytes, "amp_loss_forward")) return st;
  if (!loss_dev || (uintptr_t)loss_dev % 8) return fail(PFTPIE_E_INVALID, "amp_loss_forward: loss_dev NULL or misaligned");
  if (saved_u && (uintptr_t)saved_u % 8) return fail(PFTPIE_E_INVALID, "amp_loss_forward: saved_u misaligned");
  const size_t ub = (size_t)scan->J * scan->plan->m * scan->plan->m * 8;
  const size_t ob = (size_t)scan->H * scan->W * 8;
  if (overlaps(saved_u, ub, object, ob) || overlaps(saved_u, ub, workspace, ws_bytes) ||
      overlaps(saved_u, ub, probe, (size_t)scan->plan->n * scan->plan->n * 8))
    return fail(PFTPIE_E_INVALID, "amp_loss_forward: saved_u overlaps an input or the workspace");
  LossArgs a = base_args(scan, object, probe, amp, workspace);
  a.U = static_cast<float2*>(saved_u);
  a.loss = loss_dev;
  hipError_t e = launch_loss_forward(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "amp_loss_forward: launch");
}

pftpie_status amp_loss_backward(pie_scan scan, const void* object, const void* probe, const float* amp,
                                const void* saved_u, const double* grad_scale_dev, void* grad_object,
                                void* grad_probe, void* workspace, size_t ws_bytes, void* stream) {
  if (pftpie_status st = check_common(scan, object, probe, amp, workspace, ws_bytes, "amp_loss_backward")) return st;
  if (!grad_object) return fail(PFTPIE_E_INVALID, "amp_loss_backward: grad_object is NULL");
  if ((uintptr_t)grad_object % 8 || (grad_probe && (uintptr_t)grad_probe % 8) ||
      (saved_u && (uintptr_t)saved_u % 8) || (grad_scale_dev && (uintptr_t)grad_scale_dev % 8))
    return fail(PFTPIE_E_INVALID, "amp_loss_backward: misaligned pointer");
  const size_t ob = (size_t)scan->H * scan->W * 8, pb = (size_t)scan->plan->n * scan->plan->n * 8;
  if (overlaps(grad_object, ob, object, ob) || overlaps(grad_object, ob, probe, pb) ||
      overlaps(grad_probe, pb, object, ob) || overlaps(grad_probe, pb, probe, pb) ||
      overlaps(grad_object, ob, grad_probe, pb) || overlaps(grad_object, ob, workspace, ws_bytes) ||
      overlaps(grad_probe, pb, workspace, ws_bytes))
    return fail(PFTPIE_E_INVALID, "amp_loss_backward: gradients overlap inputs or the workspace");
  LossArgs a = base_args(scan, object, probe, amp, workspace);
  const bool recompute = (saved_u == nullptr);
  a.U = recompute ? reinterpret_cast<float2*>(workspace) : nullptr;
  a.Uc = recompute ? a.U : static_cast<const float2*>(saved_u);
  a.scale_dev = grad_scale_dev;
  a.gO = static_cast<float2*>(grad_object);
  a.gP = static_cast<float2*>(grad_probe);
  hipError_t e = launch_loss_backward(a, recompute, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PFTPIE_OK : hip_fail(e, "amp_loss_backward: launch");
}

}  // extern "C"
