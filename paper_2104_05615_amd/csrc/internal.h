// Host-side hooks shared by the library's translation units.
#pragma once

namespace mspcg {

// message returned by mspcg_last_error() on the calling thread
void set_last_error(const char* msg);

}  // namespace mspcg
