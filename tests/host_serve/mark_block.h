// Arena block marking for the host test of the served path: with the address
// sanitizer, a free block's host bytes are poisoned, so any access to a block
// outside its reservation (a queued gather or scatter that outlives it, a host
// copy after release) is reported.  Included into the server's translation unit
// by the test build.  TEST INFRASTRUCTURE ONLY.
#pragma once

#if defined(__SANITIZE_ADDRESS__)
#define SW_HS_ASAN 1
#elif defined(__has_feature)
#if __has_feature(address_sanitizer)
#define SW_HS_ASAN 1
#endif
#endif

#ifdef SW_HS_ASAN
#include <sanitizer/asan_interface.h>
#define SW_SERVE_MARK_BLOCK(p, n, live) \
  ((live) ? ASAN_UNPOISON_MEMORY_REGION((p), (n)) : ASAN_POISON_MEMORY_REGION((p), (n)))
#endif
