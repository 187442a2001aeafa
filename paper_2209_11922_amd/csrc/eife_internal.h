// Entry points shared by the library's own translation units (not part of the
// public interface in include/eife.h).
#pragma once

#include <stdint.h>

#include "../../include/eife.h"

#ifdef __cplusplus
extern "C" {
#endif

/* eife_step_out on an FP32 grid that, where its shape allows (2D, Dirichlet
 * along x, N_x = 256 or 512, the sine transforms) and u_in != u_out, also
 * writes chg[p] = sum over line pair p (rows 2p, 2p + 1) of (u_out - u_in)^2
 * in double: each of the 64 lanes adds its columns l, l + 64, ... in order
 * (row 2p, then row 2p + 1) with fused multiply-adds, then the lanes are added
 * by the butterfly over lane distances 32, 16, ..., 1.  *done = 1 when chg was
 * written, 0 when the steps ran without it.  Errors: those of eife_step_out. */
int eife_step_out_change(eife_grid g, const float* u_in, float* u_out, int64_t n_steps, int f_kind, double t0,
                         double* chg, int* done, void* stream);

#ifdef __cplusplus
}
#endif
