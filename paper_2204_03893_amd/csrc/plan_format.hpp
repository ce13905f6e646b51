// Encoding of the fused kernels' outputs, shared by the plan builder (host)
// and the kernels (device).
//
// A tile's outputs travel in 16-byte units: units rec_ptr[t] .. rec_mid[t]-1
// are pair units {target a, a0 | a1 << 16, target b, b0 | b1 << 16} holding
// two outputs of at most two entries each (unit l of the group holds outputs
// l and l + n/2, so that each store instruction covers consecutive outputs);
// the others are single units {target, c0 | c1 << 16, c2 | c3 << 16,
// c4 | c5 << 16} holding one output of at most six entries.
//
// Entries (summed in the order listed): v < carry_base(ns, T) = ns (T + 1) is
// LDS pair v of the tile's staging (symmetric pair v / (T + 1), local element
// v % (T + 1)); v >= carry_base is carry entry v - carry_base (only ever an
// output's first entry); v = T (pair 0 of the padding column, where the
// kernels keep a zero) is no entry.
//
// An output of more than six entries takes k consecutive single units that
// lie in one block of kSegLanes units of the tile (the units one wave reads in
// one round): all but the last have the code kCodeExt, and the last one, with
// the output's code, adds their sums to its own (a segmented sum across the
// wave's lanes).
//
// Target codes (int32): 0 <= code < kCodeCarry a CSR slot; kCodeCarry + k,
// k < 65536, carry entry k; kCodeExt: continued in the next unit;
// kCodeNone: a unit with no entries that stores nothing; code < 0 partial
// -(code + 1).
#pragma once

#include <cstdint>

namespace qxa {

constexpr int32_t kCodeCarry = 0x40000000;
constexpr int32_t kCodeCarryEnd = kCodeCarry + 0x10000;
constexpr int32_t kCodeExt = 0x7ffffffe;
constexpr int32_t kCodeNone = 0x7fffffff;
constexpr int kSegLanes = 64;
constexpr int kUnitEntries = 6;  // entries of a single unit
constexpr int kPairEntries = 2;  // entries of each output of a pair unit

constexpr int carry_base(int ns, int T) { return ns * (T + 1); }

}  // namespace qxa
