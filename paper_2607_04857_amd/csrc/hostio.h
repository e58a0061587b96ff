// hostio.h -- host-only file formats of the library: the tuning-cache JSON
// and the checkpoint text of sliced solves.  No HIP dependency, so the
// parsers can be built and fuzzed on their own (also under sanitizers).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "plan.h"

namespace qhost {

// ---- tuning cache (JSON)
//   {"format": "qubo-tune-1", "device": "<arch>/<CUs>cu",
//    "entries": [{"n": .., "dtype": "int32"|"fp32", "B": .., "L": ..,
//                 "tier": .., "vgpr_levels": .., "walk_ms": ..,
//                 "scope": "single"|"batch"}, ...]}
// Parse a cache text into entries; checks the format tag, the device key and
// that every entry names a plan the kernels can run (false + msg otherwise;
// entries may then hold a prefix of the file's entries).
bool parse_cache(const std::string &text, const std::string &device_key,
                 std::vector<qplan::TuneEntry> *entries, std::string *msg);
std::string format_cache(const std::vector<qplan::TuneEntry> &entries, const std::string &key);

// Whole file into *out (at most 16 MiB); false + msg on failure.
bool read_file(const char *path, std::string *out, std::string *msg);
// Write a sibling "<path>.tmp" and rename it over path.
bool write_file(const char *path, const std::string &text, std::string *msg);

// ---- checkpoint of a sliced solve (text, one field per line)
struct Ckpt {
    int n = 0;
    int dtype = 0;
    uint64_t qhash = 0;
    int A = 0, B = 0, L = 0, tier = 0, vgpr_levels = 0;
    uint64_t items = 0, next_item = 0;
    int found = 0;
    int64_t energy_i = 0;
    double energy = 0.0;
    uint64_t index = 0;
    int p = 0;
    double tol = 0.0;
    double walk_ms = 0.0;
};

// FNV-1a, 64 bit, over n, the dtype and the n*n input words.
uint64_t input_hash(const void *Q, int n, qubo_dtype_t dtype);
// Write-and-rename; false + msg on failure.
bool write_ckpt(const char *path, const Ckpt &c, std::string *msg);
// 1: read; 0: no such file; -1: unreadable or malformed (msg set).
int read_ckpt(const char *path, Ckpt *c, std::string *msg);

}  // namespace qhost
