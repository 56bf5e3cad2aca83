// Randomized / learned truncated SVD inside the two-site update.
#include "../../include/tci_c.h"
#include "runtime.hpp"
#include "tsvd.hpp"

extern "C" tci_status tci_two_site_update_sketched(tci_context ctx, int nupd, const tci_tensor* A,
                                                   const tci_tensor* B, const tci_tensor* gates,
                                                   const tci_update_params* p, tci_tensor* A_out,
                                                   tci_tensor* s_out, tci_tensor* B_out,
                                                   tci_update_info* infos) {
  (void)ctx; (void)nupd; (void)A; (void)B; (void)gates; (void)p; (void)A_out; (void)s_out; (void)B_out; (void)infos;
  TCI_RET(TCI_ERR_UNSUPPORTED, "randomized truncated SVD not built yet");
}
