// Entry points of later milestones: present so the ABI is complete.
#include "internal.hpp"

using namespace pftpie;

extern "C" {
pftpie_status pftpie_group_create(const pftpie_plan*, int32_t, const pft2d_desc*, int64_t, int64_t, int64_t,
                                  int32_t, pft2d_group* out) {
  if (out) *out = nullptr;
  return fail(PFTPIE_E_UNSUPPORTED, "grouped transform not built yet");
}
pftpie_status pftpie_group_destroy(pft2d_group) { return PFTPIE_OK; }
pftpie_status pft2d_group_run(pft2d_group, const void*, void*, void*) {
  return fail(PFTPIE_E_UNSUPPORTED, "grouped transform not built yet");
}
}
