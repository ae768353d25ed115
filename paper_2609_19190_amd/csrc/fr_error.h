// The one error message of the C ABI: the calling thread's message of its
// last failing entry point, whatever the family (map, batch, server,
// scalar).  Entry points clear it on entry and set it when they fail;
// fr_last_error() and the family-named getters all return it.
#pragma once

namespace fr {
void set_error(const char* msg);
void clear_error();
const char* last_error();
}  // namespace fr
