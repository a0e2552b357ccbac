// Run-time tiler (Section V) for the GPU kernel family: plans, their
// validity checks, and the tile-table file.
#pragma once

#include <string>
#include <vector>

#include "iaat_internal.h"

namespace iaat {

struct KidInfo {
  int fam, p1, p2, rows, cols;
};
extern const KidInfo kKids[IAAT_NUM_KIDS];

// Default plan for a (layout, m, n) sub-problem, 1 <= m, n <= 80.
PlanEntry default_plan(int layout, int m, int n);

// Fills t (kPlanCount entries) with default plans.
void build_default_table(std::vector<PlanEntry>& t);

// A plan is usable iff every kid exists, every block starts inside the
// sub-problem, blocks whose kernel does not clamp a dimension fit in it, and
// the (clipped) blocks cover the m x n exactly once.
bool check_plan(int m, int n, const PlanEntry& e, std::string* why);

// Tile-table file: header + kPlanCount entries.  Returns 0 or IAAT_ERR_TABLE.
int load_table(const char* path, std::vector<PlanEntry>& t, std::string* why);
int save_table(const char* path, const std::vector<PlanEntry>& t, std::string* why);

}  // namespace iaat
