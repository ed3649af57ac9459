// Host side of the jagged reduction's autotuner: the dataset signature, the
// cache key and the persistent cache file (JSON).  No GPU is needed except to
// read the sample of offsets that the signature is built from.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "glv.h"
#include "glv_launch.h"

namespace glv {
namespace tune {

// Event sizes read for a signature: every event when there are at most this
// many, otherwise kSampleRuns runs of consecutive events spread evenly over
// the offsets.
constexpr int64_t kSampleEvents = 65536;
constexpr int kSampleRuns = 32;

// Signature of a CSR dataset from the sizes of (a sample of) its events: the
// order of magnitude of the event count and, per size class (0; then
// [2^(b-1), 2^b) for b = 1, 2, ...), the share of the sampled events in 5 %
// steps -- e.g. "e20;3:5,4:30,5:55,6:10".  Datasets whose size distributions
// agree to within those steps share a signature.
std::string signature_of_sizes(int64_t n_events, const int64_t* sizes, int64_t n_sampled);

// The signature of device offsets (copies the sample to the host and
// synchronises `s`).
hipError_t signature(int64_t n_events, const int64_t* offsets, hipStream_t s, std::string* sig);

// Name of the current device's architecture ("gfx950"), "none" without one.
std::string arch_name();

// Cache key: architecture, dtype, coordinate system, direction and mode, and
// the dataset signature, separated by '|'.
std::string make_key(glv_dtype dt, glv_coords co, const char* what, const std::string& sig);

using Entries = std::vector<std::pair<std::string, Tiling>>;

enum class FileState { kOk, kMissing, kCorrupt };

// Reads a cache file: {"format": "glv-autotune-1", "entries": [{"key": "...",
// "tiling": [block, events_per_tile, lds_particles, pairs_per_round]}, ...]}.
// Anything else -- a syntax error, an unknown format, a duplicate key -- makes
// the file corrupt; *why names the first problem.
FileState load(const char* path, Entries* out, std::string* why);

// Writes entries to path atomically (a temporary file renamed over it);
// false on an I/O error.
bool save(const char* path, const Entries& entries);

// In-process choices by key.
bool lookup_process(const std::string& key, Tiling* t);
void remember_process(const std::string& key, const Tiling& t);
void forget_process();

}  // namespace tune
}  // namespace glv
