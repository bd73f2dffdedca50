// Error reporting shared by the C entry points.
#include <string>

#include "mhr_internal.h"

namespace mhr {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
const std::string &last_error() { return g_last_error; }

}  // namespace mhr

extern "C" const char *mhr_status_string(mhr_status s) {
    switch (s) {
        case MHR_OK: return "ok";
        case MHR_ERR_INVALID_ARGUMENT: return "invalid argument";
        case MHR_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case MHR_ERR_UNSUPPORTED: return "unsupported";
        case MHR_ERR_OUT_OF_MEMORY: return "out of memory";
        case MHR_ERR_DEVICE: return "device error";
        case MHR_ERR_NO_EMBEDDINGS: return "embeddings not set";
        case MHR_ERR_BAD_EDGE: return "edge id out of range";
        case MHR_ERR_INTERNAL: return "internal consistency check failed";
        case MHR_ERR_IO: return "file input/output error";
        case MHR_ERR_CORRUPT: return "corrupt or unrecognised file";
        case MHR_ERR_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

extern "C" const char *mhr_last_error(void) { return mhr::last_error().c_str(); }
