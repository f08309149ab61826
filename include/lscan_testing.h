/*
 * lscan_testing.h -- test hooks of liblscan.so.  Not part of the product
 * interface: they exist so that tests can reach states that a real caller
 * reaches only after billions of launches.
 *
 * Flag epochs (paper, Section 4.3 and Algorithm 4; the paper does not say
 * how its flag array is reset between scans).  Every launch tags the flag
 * words it writes with a 32-bit epoch: the kernel reads the last tag from a
 * control word, uses tag + 1, and the last workgroup to leave stores it
 * back, so no memset is needed between launches.  Before the tag could wrap
 * (after lscan_test_epoch_limit() launches on one workspace) the library
 * starts a new epoch run: it clears every flag word, restarts the tag and
 * the exit counter, and clears the word that holds the tag of the last
 * launch that gave up (a timeout), which a restarted tag could otherwise
 * meet again.  These hooks move a workspace close to that point and read its
 * state back.
 *
 * Control words of a workspace, as returned in ctrl[4]:
 *   ctrl[0]  tag of the last completed launch
 *   ctrl[1]  exit counter of the running launch (0 between launches)
 *   ctrl[2]  timeout flag (set by a launch that gave up; cleared by
 *            lscan_check / lscan_graph_check)
 *   ctrl[3]  tag of the last launch that gave up (0: none since the last
 *            epoch reset)
 */
#ifndef LSCAN_TESTING_H
#define LSCAN_TESTING_H

#include <stdint.h>

#include "lscan.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Launches one workspace may make before the library resets its epoch. */
uint64_t lscan_test_epoch_limit(void);

/*
 * Seed the flag workspace of (current device, stream): synchronize the
 * stream, clear every flag word, set the launch count to `launches`, the
 * last tag (ctrl[0]) to `tag`, the exit counter to 0 and the last-abort word
 * (ctrl[3]) to `abort_tag` (the timeout flag is kept).  With every flag word
 * cleared, no stale word can carry a tag that the seeded counter will
 * produce, so later results stay exact.  A last-abort word equal to a tag
 * that a later launch uses makes that launch give up at its first wait that
 * is not already satisfied: that is what the epoch reset must prevent.
 *   launches   <= lscan_test_epoch_limit()
 *   tag        tag + (limit - launches) + 1 < 2^32 - 1, so the seeded run
 *              reaches the reset before its tag could wrap
 *   abort_tag  any value; 0 means no launch gave up
 * LSCAN_ERR_NOT_FOUND if the stream has no workspace yet (make one scan on
 * it first); LSCAN_ERR_INVALID_ARG for values outside the ranges above.
 */
lscan_status lscan_test_seed_epoch(void *stream, uint64_t launches,
                                   uint32_t tag, uint32_t abort_tag);

/* The same for the workspace a captured graph owns (synchronizes the
 * device first). */
lscan_status lscan_test_graph_seed_epoch(lscan_graph *g, uint64_t launches,
                                         uint32_t tag, uint32_t abort_tag);

/*
 * Read back the launch count and control words 0..3 of the workspace of
 * (current device, stream) after synchronizing the stream.
 * LSCAN_ERR_NOT_FOUND if the stream has no workspace.
 */
lscan_status lscan_test_epoch_state(void *stream, uint64_t *launches,
                                    uint32_t ctrl[4]);

/* The same for a graph's workspace (synchronizes the device first). */
lscan_status lscan_test_graph_epoch_state(lscan_graph *g, uint64_t *launches,
                                          uint32_t ctrl[4]);

#ifdef __cplusplus
}
#endif

#endif /* LSCAN_TESTING_H */
