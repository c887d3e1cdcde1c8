// Internal declarations shared by the library's translation units.
#ifndef NZE_INTERNAL_H
#define NZE_INTERNAL_H

#include <string>

namespace nze {

// Records msg as the calling thread's last error and returns code.
int fail(int code, const char* msg);

extern thread_local std::string g_last_error;

}  // namespace nze

#endif
