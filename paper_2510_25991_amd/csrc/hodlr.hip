// Compressed (weak-admissibility hierarchical) form of the transfer blocks.
#include "internal.h"

namespace ddst {
void hodlr_free(ddst_op *op) { (void)op; }
bool hodlr_ready(const ddst_op *op) { return op && op->hodlr != nullptr; }
int hodlr_compress(ddst_op *, const ddst_compress_opts_t &, hipStream_t) { return DDST_ESTATE; }
int hodlr_apply_jobs(const ddst_op *, const double *, double *, int, hipStream_t) {
  return DDST_ESTATE;
}
}  // namespace ddst

extern "C" int ddst_compress(ddst_op_t *op, const ddst_compress_opts_t *opts, hipStream_t s) {
  if (!op || !opts) return DDST_EINVAL;
  return ddst::hodlr_compress(op, *opts, s);
}
