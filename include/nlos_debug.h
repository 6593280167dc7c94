/*
 * nlos_debug.h -- test hooks of libnlos (not needed by applications).
 */
#ifndef NLOS_DEBUG_H
#define NLOS_DEBUG_H

#ifdef __cplusplus
extern "C" {
#endif

/* Makes the next n allocations of the library fail as if memory were exhausted: device
 * allocations (plan tables, the context's workspace pool and tables) and host allocation
 * points (plan and kernel construction).  The call that meets one returns
 * NLOS_ERR_OUT_OF_MEMORY with nothing enqueued and nothing leaked, and the context stays
 * usable.  n = 0 clears the injection.  Process wide; for fault-path tests. */
void nlos_debug_fail_allocations(int n);

#ifdef __cplusplus
}
#endif

#endif /* NLOS_DEBUG_H */
