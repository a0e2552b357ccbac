// Run-time tiler for the GPU kernel family.
//
// The paper's tiler (Section V-A, Algorithm 2) cuts C into row strips whose
// heights are kernel sizes, cuts each strip's N into kernel widths, and picks
// between candidate cuttings by the number of loads from cache to registers,
// (sum_i (m_i + n_i)) K + 2MN ("Minimal Memops"), preferring bigger blocks.
// The GPU family differs (a block is what one 64-lane wavefront computes), so
// the default plan here is the GPU reading of the same principles:
//   * tiny m x n (both <= 4): one K-split block (all 64 lanes share K);
//   * m <= 8: one row strip of height m, cut into 64-column pieces;
//   * n <= 8: one column strip of width n, cut into 64-row pieces;
//   * otherwise matrix-core tiles: ceil(m/16) x ceil(n/16) 16x16 tiles,
//     split into at most two balanced groups per dimension (1 -> 1,
//     2 -> 1+1, 3 -> 2+1, 4 -> 2+2, 5 -> 3+2), so a sub-problem has at most
//     four blocks of at most 3 x 3 tiles: one block per wavefront of the
//     batched kernel's work-group, which reads A and B from LDS, so the
//     extra block edges (sum(m_i + n_i) grows with the block count) cost
//     LDS reads rather than memory traffic.
// The plan depends only on (layout, m, n), never on K: every candidate
// moves K * sum(m_i + n_i) operand values, so K does not change the order.
// The autotuner may replace any plan with one it measured faster; every plan
// is checked by check_plan before use.
#include "tiler.h"

#include <stdio.h>
#include <string.h>

namespace iaat {

const KidInfo kKids[IAAT_NUM_KIDS] = {
#define IAAT_INFO(id, fam, p1, p2, br, bc) {fam, p1, p2, br, bc},
    IAAT_FOR_EACH_KID(IAAT_INFO)
#undef IAAT_INFO
};

static int find_kid(int fam, int p1, int p2) {
  for (int i = 0; i < IAAT_NUM_KIDS; ++i)
    if (kKids[i].fam == fam && kKids[i].p1 == p1 && kKids[i].p2 == p2) return i;
  return -1;
}

// Split t <= 6 tiles into at most two groups, as evenly as possible.
static int split_tiles(int t, int* sizes) {
  const int g = t > 1 ? 2 : 1;
  for (int i = 0; i < g; ++i) sizes[i] = t / g + (i < t % g ? 1 : 0);
  return g;
}

PlanEntry default_plan(int layout, int m, int n) {
  (void)layout;
  PlanEntry e;
  memset(&e, 0, sizeof e);
  if (m <= 4 && n <= 4) {
    e.blk[e.nblk++] = pack_block(0, 0, find_kid(FAM_KRED, m, n));
  } else if (m <= 8) {
    const int kid = find_kid(FAM_ROWS, m, 64);
    for (int j0 = 0; j0 < n; j0 += 64) e.blk[e.nblk++] = pack_block(0, j0, kid);
  } else if (n <= 8) {
    const int kid = find_kid(FAM_COLS, 64, n);
    for (int i0 = 0; i0 < m; i0 += 64) e.blk[e.nblk++] = pack_block(i0, 0, kid);
  } else {
    int gm[8], gn[8];
    const int ngm = split_tiles((m + 15) / 16, gm), ngn = split_tiles((n + 15) / 16, gn);
    int r0 = 0;
    for (int a = 0; a < ngm; ++a) {
      int c0 = 0;
      for (int b = 0; b < ngn; ++b) {
        e.blk[e.nblk++] = pack_block(16 * r0, 16 * c0, find_kid(FAM_MFMA, gm[a], gn[b]));
        c0 += gn[b];
      }
      r0 += gm[a];
    }
  }
  return e;
}

void build_default_table(std::vector<PlanEntry>& t) {
  t.assign(kPlanCount, PlanEntry{});
  for (int lay = 0; lay < kLayouts; ++lay)
    for (int m = 1; m <= kSuper; ++m)
      for (int n = 1; n <= kSuper; ++n) t[plan_index(lay, m, n)] = default_plan(lay, m, n);
}

bool check_plan(int m, int n, const PlanEntry& e, std::string* why) {
  char msg[160];
  if (e.nblk < 1 || e.nblk > (uint32_t)kMaxBlocks) {
    snprintf(msg, sizeof msg, "plan %dx%d: %u blocks", m, n, e.nblk);
    if (why) *why = msg;
    return false;
  }
  unsigned char cover[kSuper][kSuper];
  memset(cover, 0, sizeof cover);
  for (uint32_t b = 0; b < e.nblk; ++b) {
    const int i0 = blk_i0(e.blk[b]), j0 = blk_j0(e.blk[b]), kid = blk_kid(e.blk[b]);
    if (kid >= IAAT_NUM_KIDS || i0 >= m || j0 >= n) {
      snprintf(msg, sizeof msg, "plan %dx%d block %u: kid %d at (%d,%d)", m, n, b, kid, i0, j0);
      if (why) *why = msg;
      return false;
    }
    const KidInfo& k = kKids[kid];
    // the row strip does not clamp rows, the column strip does not clamp
    // columns, the K-split block clamps neither
    const bool rows_exact = k.fam == FAM_ROWS || k.fam == FAM_KRED;
    const bool cols_exact = k.fam == FAM_COLS || k.fam == FAM_KRED;
    if ((rows_exact && i0 + k.rows > m) || (cols_exact && j0 + k.cols > n)) {
      snprintf(msg, sizeof msg, "plan %dx%d block %u: kid %d overruns", m, n, b, kid);
      if (why) *why = msg;
      return false;
    }
    const int ie = i0 + k.rows < m ? i0 + k.rows : m, je = j0 + k.cols < n ? j0 + k.cols : n;
    for (int j = j0; j < je; ++j)
      for (int i = i0; i < ie; ++i)
        if (cover[i][j]++) {
          snprintf(msg, sizeof msg, "plan %dx%d: (%d,%d) covered twice", m, n, i, j);
          if (why) *why = msg;
          return false;
        }
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i)
      if (!cover[i][j]) {
        snprintf(msg, sizeof msg, "plan %dx%d: (%d,%d) not covered", m, n, i, j);
        if (why) *why = msg;
        return false;
      }
  return true;
}

namespace {
struct TableHeader {
  char magic[8];
  uint32_t version;
  uint32_t family_hash;
  uint32_t nplans;
  uint32_t entry_bytes;
  char arch[16];
  uint32_t reserved[4];
};
const char kMagic[8] = {'I', 'A', 'A', 'T', 'T', 'B', 'L', '1'};
}  // namespace

int load_table(const char* path, std::vector<PlanEntry>& t, std::string* why) {
  FILE* f = fopen(path, "rb");
  if (!f) {
    if (why) *why = std::string("cannot open tile table ") + path;
    return IAAT_ERR_TABLE;
  }
  TableHeader h;
  std::vector<PlanEntry> tmp(kPlanCount);
  const bool ok = fread(&h, sizeof h, 1, f) == 1 &&
                  fread(tmp.data(), sizeof(PlanEntry), kPlanCount, f) == (size_t)kPlanCount;
  fclose(f);
  if (!ok || memcmp(h.magic, kMagic, 8) != 0 || h.version != 1 ||
      h.nplans != (uint32_t)kPlanCount || h.entry_bytes != sizeof(PlanEntry)) {
    if (why) *why = std::string("not a tile table: ") + path;
    return IAAT_ERR_TABLE;
  }
  if (h.family_hash != IAAT_FAMILY_HASH || strncmp(h.arch, "gfx950", sizeof h.arch) != 0) {
    if (why) *why = std::string("tile table built for another kernel family or arch: ") + path;
    return IAAT_ERR_TABLE;
  }
  for (int lay = 0; lay < kLayouts; ++lay)
    for (int m = 1; m <= kSuper; ++m)
      for (int n = 1; n <= kSuper; ++n)
        if (!check_plan(m, n, tmp[plan_index(lay, m, n)], why)) return IAAT_ERR_TABLE;
  t.swap(tmp);
  return 0;
}

int save_table(const char* path, const std::vector<PlanEntry>& t, std::string* why) {
  TableHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, kMagic, 8);
  h.version = 1;
  h.family_hash = IAAT_FAMILY_HASH;
  h.nplans = kPlanCount;
  h.entry_bytes = sizeof(PlanEntry);
  strncpy(h.arch, "gfx950", sizeof h.arch - 1);
  FILE* f = fopen(path, "wb");
  if (!f) {
    if (why) *why = std::string("cannot write ") + path;
    return IAAT_ERR_TABLE;
  }
  const bool ok = fwrite(&h, sizeof h, 1, f) == 1 &&
                  fwrite(t.data(), sizeof(PlanEntry), t.size(), f) == t.size();
  fclose(f);
  if (!ok) {
    if (why) *why = std::string("short write to ") + path;
    return IAAT_ERR_TABLE;
  }
  return 0;
}

}  // namespace iaat
