// Per-bin kernel configuration for gfx950 (CDNA4), shared by host and device.
//
// The paper sizes each bin's hash table so that every kernel reaches full
// occupancy (Section 5.6): on V100 that is 96 KB shared memory for 2048
// threads.  On gfx950 a compute unit has 160 KB of LDS and holds at most
// 32 waves of 64 lanes (2048 lanes), i.e. 80 B of LDS per lane at full
// occupancy; the tables below follow that rule, with the last LDS bin of
// each step deliberately at 50 % occupancy to use all 160 KB (as the paper
// does with its largest shared-memory bin).
#pragma once

#include <stdint.h>

namespace opsp {

// ---- symbolic step: int32 keys -------------------------------------------
// bin 0: several rows per wave, SYM_GL lanes per row (tiny rows)
// bin 1: one wave per row (4 rows per 256-lane workgroup)
// bins 2..7: one workgroup per row; bin 7 abandons rows whose distinct count
// crosses the abort threshold, and those rows are redone with global tables.
constexpr int SYM_GL = 8;
constexpr int SYM_NLDS = 8;
constexpr int SYM_T[SYM_NLDS] = {128, 1024, 2048, 4096, 8192, 16384, 20448, 40896};
constexpr int SYM_W[SYM_NLDS] = {SYM_GL, 64, 128, 256, 512, 1024, 1024, 1024};
constexpr int SYM_GLOBAL_BIN = 8;

// ---- numeric step: (int32 key, double value) entries ----------------------
constexpr int NUM_GL = 8;
constexpr int NUM_NLDS = 7;
constexpr int NUM_T[NUM_NLDS] = {39, 425, 848, 1700, 3408, 6816, 13632};
constexpr int NUM_W[NUM_NLDS] = {NUM_GL, 64, 128, 256, 512, 1024, 1024};
constexpr int NUM_GLOBAL_BIN = 7;

// Bin 0 packs several rows into one 256-lane workgroup with GROUP_GL[v]
// lanes and a table of SYM_T0[v] / NUM_T0[v] entries per row; the variants
// keep the workgroup's LDS the same (fewer lanes, more and smaller rows).
// Variant 0 is the default; config.group_lanes selects another.
constexpr int GROUP_VARIANTS = 3;
constexpr int GROUP_GL[GROUP_VARIANTS] = {SYM_GL, 4, 16};
constexpr int SYM_T0[GROUP_VARIANTS] = {SYM_T[0], 64, 256};
constexpr int NUM_T0[GROUP_VARIANTS] = {NUM_T[0], 19, 79};
static_assert(SYM_GL == NUM_GL, "one lane count for both steps");
// Variant of a lane count (0 = default), -1 when there is none.
constexpr int group_variant(int lanes) {
    return lanes == 0 || lanes == GROUP_GL[0] ? 0 : lanes == GROUP_GL[1] ? 1 : lanes == GROUP_GL[2] ? 2 : -1;
}

// Workgroups per CU that the global-table kernels are sized for.
constexpr int SYM_GLOBAL_WG_PER_CU = 1;

// B-row entries each lane of a several-rows-per-wave kernel loads before it
// inserts them (loads in flight per lane).
constexpr int GRP_U = 8;

// Symbolic rows of the global bin with a known column range are counted in
// an LDS bitmap of 2^SW_LG columns, one pass per window of the range, when
// the range needs at most SW_MAXPASS windows.
constexpr int SW_LG = 20;

// Windows of B loads in flight per wave beyond the current one in the
// kernels that give a row 512 or more threads (long rows: few waves per CU
// to hide the load latency).
constexpr int WIDE_D = 2;
// ... and in the symbolic bin-7 kernel, which has the CU to itself (all of
// the LDS; four waves per SIMD leave it 128 vector registers)
constexpr int SYM_ABORT_D = 6;
constexpr int SW_MAXPASS = 8;
constexpr int NUM_GLOBAL_WG_PER_CU = 1;

// Columns per LDS bitmap chunk used to order a global-table row.
constexpr int NUM_GLOBAL_CHUNK_WORDS = 16384;   // 2^19 columns, 64 KB

}  // namespace opsp
