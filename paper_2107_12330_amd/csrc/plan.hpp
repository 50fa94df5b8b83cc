// plan.hpp -- sizes shared by the survey planner (build) and the survey
// kernels.
#pragma once

#include <cstdint>

namespace tp {

// Targets q are split into classes by d+(q): the class decides how Adj+(q)
// is searched.  Tiny, small and large targets keep a two-table cuckoo hash
// of Adj+(q) in LDS (each table 2^k >= 1.25 d+(q) slots, so the load stays
// at most 0.4, plus a small stash); tiny ones get one table per wave, small
// and large ones one per workgroup; huge ones are searched in HBM.
constexpr uint32_t kTinyMaxDeg = 51;     // per-wave tables of <= 64 slots
constexpr uint32_t kSmallMaxDeg = 819;   // tables of <= 1024 slots
constexpr uint32_t kLargeMaxDeg = 3276;  // tables of <= 4096 slots
constexpr int kTinyLogSlots = 6;
constexpr int kSmallLogSlots = 10;
constexpr int kLargeLogSlots = 12;
constexpr uint32_t kStash = 32;          // keys the cuckoo insertion could not place

// A tile holds at most `cap` in-edge records of one target and about
// kTileWorkPerRecord * cap wedge checks.  Default caps per target class:
// 1024 records, and 16384 for the large class, whose workgroups stall for
// the first records of every tile; the tuner may choose others.
constexpr uint32_t kTileRecords = 1024;
constexpr uint64_t kTileWorkPerRecord = 256;
inline uint32_t default_tile_records(int cls) { return cls == 2 ? 16384u : kTileRecords; }

// Slots of padding after the last oriented edge in the target and time
// arrays, so that a wave may load 64 consecutive slots from any row start.
constexpr uint64_t kRowPad = 64;

}  // namespace tp
