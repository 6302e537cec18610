// Device primitives: scans, LSD radix sort, segmented min/max, fills.
#pragma once

#include "pool.h"

namespace jp {

// out[0..n] = exclusive prefix sums of in[0..n); out[n] = total.
void scan_excl_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s, Arena& a);
void scan_excl_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s, Arena& a);
void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s, Arena& a);

// Input already grouped by segment: segment i holds elements [ebase[i],
// ebase[i+1]) (device and host copies) and its keys lie in [koff[i],
// koff[i] + 2^bits).
struct SortSegments {
  int n_seg;
  const int32_t* d_ebase;             // [n_seg + 1]
  const int64_t* d_koff;              // [n_seg]
  const std::vector<int32_t>& h_ebase;  // [n_seg + 1]
};

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys, or, with segments, of every segment in place on the low `bits` bits of
// key - koff[i] (passes then depend on the widest segment's key range, not on
// the stacked ranges).  The sorted data ends up either in (k, v) or in
// (kt, vt); the function returns true when it is in (kt, vt).  `v` may be null
// (keys only).
bool radix_sort_pairs(uint32_t* k, uint32_t* v, uint32_t* kt, uint32_t* vt, int64_t n, int bits,
                      hipStream_t s, Arena& a, const SortSegments* seg = nullptr);
// passes radix_sort_pairs makes (an odd count leaves the data in (kt, vt))
int radix_passes(int64_t n, int bits);
// radix_sort_pairs of the keys koff[i] + raw - mn[i] of raw int32 values
// grouped by segment, with raw_v (or nothing, if null) as their values: the
// first pass reads (raw, raw_v) and makes the keys as it loads them, the rest
// ping-pong between (kt, vt) and (k, v) as radix_sort_pairs does, so the
// result lies where radix_sort_pairs would leave it.  With seg_raw (device
// array of n_seg pointers, more than one segment), the raw values of segment
// i are read from their own buffer seg_raw[i] (values seg_raw_v[i]) and raw,
// raw_v are not used.  Needs at least one pass (radix_passes(n, bits) > 0).
bool radix_sort_raw(const int32_t* raw, const int32_t* raw_v, const int32_t* const* seg_raw,
                    const int32_t* const* seg_raw_v, const int32_t* mn, uint32_t* k, uint32_t* v, uint32_t* kt,
                    uint32_t* vt, int64_t n, int bits, hipStream_t s, Arena& a, const SortSegments& seg);

// Per-segment min and max of int32 values; segment i is [base[i], base[i+1]).
// mn/mx (n_seg entries) are overwritten; empty segments give mn > mx.
void seg_minmax(const int32_t* v, int64_t n, const int32_t* base, int n_seg, int32_t* mn,
                int32_t* mx, hipStream_t s);

void fill_i32(int32_t* p, int64_t n, int32_t val, hipStream_t s);
void fill_i64(int64_t* p, int64_t n, int64_t val, hipStream_t s);
void fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t s);

// Sum of a[0..n) into *out (int64, device).
void reduce_sum_i32_to_i64(const int32_t* a, int64_t n, int64_t* out, hipStream_t s);

int bits_for(uint64_t range);  // number of bits to hold values in [0, range)

}  // namespace jp
