// admm_host.h — host-only logic of the library (no HIP, no device): error
// messages, the plan-time validation of a problem, and the autotuner's JSON
// cache. Kept apart from the HIP sources so that it can also be built on its
// own with the address and undefined-behaviour sanitizers (tests/).
#pragma once
#include <map>
#include <string>

#include "../../include/admm_deconv.h"

#ifndef ADMM_MAX_SIDE
#define ADMM_MAX_SIDE 16384
#endif

namespace admm_host {

// Set the calling thread's error message (printf-style) and return s.
admm_status fail(admm_status s, const char* fmt, ...);
// The calling thread's last error message.
const char* last_error();
// Prefix the calling thread's error message (e.g. with the problem index).
void prefix_error(const std::string& prefix);

// n = 2^a 3^b 5^c 7^d with n >= 1 (the transform lengths the library plans)
bool smooth7(int n);

// Plan-time checks of one problem (sides, kernel, regulariser, parameters).
admm_status validate(const admm_problem& p);

// One cache entry: columns per column block, rows per row block (and per
// size class of the row length: 0 = use rows), the radix schedule variants
// ("rsched", "csched"; written when not 0) and the per-launch timings of the
// choice, for the record.
constexpr double kMaxTileCount = 4096.0;
constexpr int kRowClasses = 6;   // size classes of the row length: <= 512, 1024, 2048, 4096, 8192, 16384
struct TuneEntry {
    int tc = 0, rows = 0;
    int rows_c[kRowClasses] = {};   // "rows_512", "rows_1024", ..., "rows_16384"
    int rsched = 0, csched = 0;  // radix schedule variants of the row and column transforms
    double col_us = 0.0, row_us = 0.0;
};
constexpr int kScheduleVariants = 4;

// Parse the cache text; false if it is not an object of objects of numbers
// with valid values.
bool parse_cache(const std::string& text, std::map<std::string, TuneEntry>& out);
std::string format_cache(const std::map<std::string, TuneEntry>& m);
// 0: read (or absent: empty map); -1: unreadable or malformed
int read_cache(const char* path, std::map<std::string, TuneEntry>& out);
// 0: written (atomically, through a temporary file); -1: failed
int write_cache(const char* path, const std::map<std::string, TuneEntry>& m);
// "<arch>|<shape multiset>" (a hash of the list for long ragged batches)
std::string make_key(const admm_problem* probs, int count, const char* arch);

}  // namespace admm_host
