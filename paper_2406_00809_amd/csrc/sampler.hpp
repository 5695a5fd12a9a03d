// Training-pair sampler of Sec. 2.2 (Eqs. (2)-(3)); internal interface used
// by the training loop.  The C entry points are declared in gnp.h.
#pragma once
#include "gnp_internal.hpp"

namespace gnp {

// m unpreconditioned Arnoldi steps from xi ~ N(0, I) (seed, stream 2), SVD
// of Hbar, G = Z S^+.  max_count: most draws per call.  Synchronises st.
gnp_status sampler_create(gnp_system *sys, int m, uint64_t seed, int max_count, hipStream_t st,
                          gnp_sampler **out);
void sampler_destroy(gnp_sampler *sp);

// Columns d = 0..count-1 of x ([n][B], element type T) receive draw d of
// training step `step`: x = V_m G eps_d, eps_d from stream 1 (element
// d * k + j).  Enqueued on st.
template <typename T>
gnp_status sampler_draw_launch(gnp_sampler *sp, uint32_t step, int count, int B, T *x,
                               hipStream_t st);

}  // namespace gnp
