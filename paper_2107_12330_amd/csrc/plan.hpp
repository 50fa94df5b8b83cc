// plan.hpp -- sizes shared by the survey planner (build) and the survey
// kernels.
#pragma once

#include <cstdint>

namespace tp {

// Targets q are split into classes by d+(q): the class decides how Adj+(q)
// is searched.  Small and large targets keep an open-addressing hash of
// Adj+(q) in LDS with at most 50% load; huge ones are searched in HBM.
constexpr uint32_t kSmallMaxDeg = 1024;  // hash of <= 2048 slots
constexpr uint32_t kLargeMaxDeg = 4096;  // hash of <= 8192 slots
constexpr int kSmallLogSlots = 11;
constexpr int kLargeLogSlots = 13;

// A tile holds at most kTileRecords in-edge records of one target and about
// kTileWork wedge checks.
constexpr uint32_t kTileRecords = 512;
constexpr uint64_t kTileWork = 65536;

}  // namespace tp
