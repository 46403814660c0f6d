/*
 * pds_testing.h -- test hooks of libpds, not part of the inference API.
 *
 * The library exports these two functions so that its tests can reach code
 * paths and launch decisions that ordinary inputs reach only rarely or not
 * observably.  Inference callers need neither.
 */
#ifndef PDS_TESTING_H
#define PDS_TESTING_H

#include "pds.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Testing aid: moves the sampled median bracket of later svgd_phi calls by
 * `ranks` sample positions (default 0), so tests can make it miss the
 * middle ranks and exercise the exact recovery pass.  The bandwidth stays
 * exact for every value; only the time changes.  Process-wide, not
 * synchronised with calls in flight.  PDS_EINVAL if |ranks| > 1e6. */
int pds_test_median_shift(int32_t ranks);

/* Test hook (host logic only, no device access): the launch shape
 * sim_batch_adjoint gives a planar job (PDS_MODEL_PLANAR or
 * PDS_MODEL_PLANAR_RIGID), read from the shape fields of *h_job (model,
 * n_dof, N, K, n_s, h).  Returns bit 0 = two lanes per window unit (the job
 * has fewer waves than the chip has SIMDs), bit 1 = the whole window in LDS
 * (else sqrt(h) checkpoints), bit 2 = the dynamics tape in LDS as well (two
 * point-mass links); writes the block's dynamic LDS bytes to *lds_bytes.
 * PDS_EINVAL for a null argument, another model or a non-positive size. */
int pds_test_adjoint_shape(const pds_job* h_job, size_t* lds_bytes);

#ifdef __cplusplus
}
#endif

#endif /* PDS_TESTING_H */
