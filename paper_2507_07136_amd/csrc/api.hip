// Status strings and version of libls2.
#include "ls2_internal.h"

extern "C" const char* ls2_status_string(int status) {
    switch (status) {
        case LS2_OK: return "ok";
        case LS2_ERR_ARG: return "invalid argument";
        case LS2_ERR_CAPACITY: return "pair capacity exceeded";
        case LS2_ERR_UNSUPPORTED: return "unsupported shape";
        case LS2_ERR_DEVICE: return "HIP device error";
        default: return "unknown status";
    }
}

extern "C" int ls2_version(void) { return 100; }

#ifndef LS2_SOURCE_HASH
#define LS2_SOURCE_HASH "unknown"
#endif
extern "C" const char* ls2_source_hash(void) { return LS2_SOURCE_HASH; }
