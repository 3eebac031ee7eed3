// Context only, not part of the oracle: the C++ standard library's
// std::sort of int32 keys, single-threaded, for timing the oracle against a
// common library sort on the same inputs.  Test infrastructure: shares no
// code with the GPU library.
#include <algorithm>
#include <cstdint>

extern "C" void context_std_sort_i32(int32_t *a, int64_t n) { std::sort(a, a + n); }
