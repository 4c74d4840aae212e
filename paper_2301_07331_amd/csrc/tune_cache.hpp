// tune_cache.hpp -- the autotuner's cache: tuned values per workload bucket,
// kept in memory and, when $HLC_TUNE_CACHE names a file, in a flat JSON
// object {"bucket": [v0, v1, ...], ...}. A bucket names the device (gfx
// architecture and compute-unit count) as well as the workload's size class,
// so values tuned on one device are never reused on another.
#pragma once

#include <string>
#include <vector>

namespace hlc {

// the cached values of a bucket, or false
bool tune_lookup(const std::string& bucket, std::vector<double>* values);
// records (and, with $HLC_TUNE_CACHE, writes out) a bucket's values
void tune_store(const std::string& bucket, const std::vector<double>& values);
// "<gfx arch>|cu<count>" of the current device
std::string tune_device_tag();

}  // namespace hlc
