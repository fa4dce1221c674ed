// Library-internal helpers shared by the host translation units.
#pragma once

namespace m1 {
// Sets the calling thread's m1_last_error() message; returns code.
int record_error(int code, const char* msg);
}  // namespace m1
