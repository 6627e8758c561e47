/*
 * rbp_test.h -- test hooks of librbp.  Not part of the decoding interface:
 * these calls exist so that tests can force rare paths from the host, and no
 * product code calls them.
 */
#ifndef RBP_TEST_H_
#define RBP_TEST_H_

#include "rbp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Latency mode (rbp_decode_coop) on this handle: its grid barriers also wait
 * for `phantom` (0..1024) workgroups that never arrive, so every barrier wait
 * runs into its poll bound and the launch stops with RBP_ERR_ABORTED.  This
 * exercises the expiry path without any kernel hanging; 0 restores normal
 * launches. */
rbp_status rbp_test_set_coop_phantom(rbp_code_t code, int32_t phantom);

#ifdef __cplusplus
}
#endif
#endif /* RBP_TEST_H_ */
