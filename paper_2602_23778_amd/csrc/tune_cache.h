// Persistent store of the launch-configuration tuners' choices (host code).
//
// With REFINE_TUNE_CACHE=<file> set, a tuner first looks its key up in the
// process's table, then in the file (read once per process), and appends
// every new choice to the file, so that later processes skip the timing
// sweep.  Each line is "<arch> <kind> <key...> : <value...>"; arch is the
// device's architecture name, so one file can serve several GPU models.
// Without the variable the table lives only as long as the process.
#pragma once
#include <stdint.h>

#include <vector>

namespace rfk {

bool tune_cache_get(const char* kind, const std::vector<int64_t>& key, std::vector<int>* value);
void tune_cache_put(const char* kind, const std::vector<int64_t>& key,
                    const std::vector<int>& value);

}  // namespace rfk
