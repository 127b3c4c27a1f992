// Thread-local error message shared by every entry point of the library.
#pragma once
#include <string>

namespace me {
void set_error(const std::string& msg);
}  // namespace me
