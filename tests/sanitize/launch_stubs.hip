// Host-only stand-ins for the kernel launchers, so that the C ABI's host
// code (argument checks, layout arithmetic, error paths) can be built and
// run with AddressSanitizer / UndefinedBehaviorSanitizer on a machine
// without a GPU (tests/test_sanitizers.py).  None of them is reached there:
// sts_create fails before any launch when no device is present.
#include "../../paper_1802_04243_amd/csrc/sts_internal.h"

namespace sts {
void launch_prologue(const Params &, State, Consts, int, hipStream_t) {}
void launch_pass(const Params &, State, State, Consts, int, const Resid *, const Inter *,
                 hipStream_t) {}
void launch_pass_first(const Params &, State, State, Consts, int, hipStream_t) {}
void launch_pass3(const Params &, State, State, Consts, int, const Resid *, int, const double *,
                  const double *, double *, double *, hipStream_t) {}
void launch_residual(const Params &, State, Consts, Resid, double *, hipStream_t) {}
void launch_loop2_reset(int *, hipStream_t) {}
void launch_loop2_check(const Params &, Resid, double *, const Loop2 &, hipStream_t) {}
void launch_loop2_final(const Params &, State, State, Consts, Resid, double *, const int *,
                        hipStream_t) {}
void launch_adjoint_pass(const Params &, State, Consts, Inter, State, State, Consts, AdjTmp,
                         double *, double *, int, hipStream_t) {}
void launch_cell_cache(const Params &, State, double *, double *, hipStream_t) {}
void launch_adjoint_prologue(const Params &, State, Consts, State, AdjTmp, int, hipStream_t) {}
int drag_blocks(const Params &) { return 1; }
void launch_drag(const Params &, State, double *, double *, hipStream_t) {}
void launch_drag_seed(const Params &, State, State, double, hipStream_t) {}
}  // namespace sts
