// lm_plan.hip -- launch plans of the pair sums (host code): how many source splits the
// one-sided kernel gets, and whether and how wide the symmetric kernels run.
#include <stdint.h>
#include <stdlib.h>

#include "lm_internal.h"

namespace lm {

PairPlan plan_pair(int64_t nt, int64_t ns, bool cut, bool sym_ok, int kind)
{
    PairPlan pl{};
    pl.itiles = (nt + kTile - 1) / kTile;
    // tile skipping runs symmetric (sums with forces) by the size rule only from kSymCutTiles
    // tiles: with much skipped, the symmetric kernel's fixed costs (superblock tests, the
    // flags, the finish) need a large N to pay off
    if (sym_ok && nt == ns && (!cut || kind == SYM_F64 || kind == SYM_F32)) {
        const char* e = getenv("LM_SYM");
        const int mode = e ? atoi(e) : -1;
        const bool small_cut = cut && mode != 1 && pl.itiles < kSymCutTiles;
        if (mode != 0 && !small_cut) {
            const SymPlan sp = plan_sym(nt, mode == 1, kind, cut);
            if (sp.waves > 0) {
                pl.sym_waves = sp.waves;
                pl.sym_rows = sp.rows;
                pl.sym_nsb = sp.nsb;
                pl.nsplit = (int)(sp.nsb + 1);
                pl.jchunk = ns;
                return pl;
            }
        }
    }
    // aim for >= LM_MIN_GROUPS workgroups (the targets alone give nt/64; the sources are
    // split over grid-y to make up the rest) while keeping every wave's chunk >= 32 sources
    int64_t s = (LM_MIN_GROUPS + pl.itiles - 1) / pl.itiles;
    int64_t smax = ns / (kWaves * 32);
    if (smax < 1) smax = 1;
    if (s > smax) s = smax;
    if (s > 64) s = 64;
    // from 80 target tiles (N = 5120) on, more than 16 splits only shortens the chunks and
    // lengthens the finish: measured at N = 16384, 3-D, FP64, 16 splits beat 64 by 12%
    // (Gaussian) and 4% (conon); at N = 6000 (94 tiles) 16 beat 46 by 10%, while at N = 4096
    // (64 tiles, 2-D) 32 beat 16 by 3%
    if (pl.itiles >= 80 && s > 16) s = 16;
    if (s < 1) s = 1;
    pl.nsplit = (int)s;
    int64_t chunks = (int64_t)pl.nsplit * kWaves;
    pl.jchunk = (ns + chunks - 1) / chunks;
    if (cut) pl.jchunk = (pl.jchunk + kTile - 1) / kTile * kTile;   // chunks start on tile boundaries
    return pl;
}

SymPlan plan_sym(int64_t n, bool force, int kind, bool cut)
{
    SymPlan sp{};
    const int64_t T = tiles_of(n);
    // LM_SYM_WAVES fixes the workgroup width and LM_SYM_ROWS the row tiles per wave (tuning
    // runs, tests of every shape); four rows exist for sums with forces and without cutoff
    const char* env = getenv("LM_SYM_WAVES");
    const int fixed = env ? atoi(env) : 0;
    const char* env_rows = getenv("LM_SYM_ROWS");
    const int fixed_rows = env_rows ? atoi(env_rows) : 0;
    const bool wide_ok = (kind == SYM_F64 || kind == SYM_F32) && !cut;
    int rows = kSymRows;
    int w = 0;
    if (fixed == 1 || fixed == 2 || fixed == 4 || fixed == 8) {
        w = fixed;
        // (at most four waves: sums without forces fall back to two rows and twice the waves)
        if (wide_ok && fixed_rows == kSymRowsWide && fixed <= 4) rows = kSymRowsWide;
    } else if (kind == SYM_VJP) {
        w = T >= kSymVjpTwoWaveTiles ? 2 : T >= kSymVjpMinTiles ? 1 : 0;
    } else if (kind == SYM_F64 && T >= kSymWideTiles) {
        // all pairs: superblocks of 8 tiles, four rows and two waves. With tile skipping,
        // superblocks of 4 tiles (two rows, two waves): a workgroup lasts as long as its
        // busiest wave, and the narrower superblocks spread the near tile pairs more evenly
        // (3-D Gaussian N = 65536 shoot 158 ms against 190 ms with 8-tile superblocks)
        rows = (wide_ok && fixed_rows != kSymRows) ? kSymRowsWide : kSymRows;
        w = cut ? 2 : 8 / rows;
    } else if (kind == SYM_F32 && T >= kSymMinTilesF32) {
        // with tile skipping superblocks of 4 tiles, as in double precision
        if (cut)
            w = 2;
        else
            w = T >= kSymF32FourWaveTiles ? 4 : T >= kSymF32TwoWaveTiles ? 2 : 1;
    } else if (kind == SYM_F64 && T >= kSymMinTiles) {
        w = 2;
    } else if (kind == SYM_F64 && T >= kSymOneWaveTiles) {
        w = 1;
    }
    if (w == 0 && force) w = 1;
    if (w == 0) return sp;
    // partial sums: (S + 1) slots of up to 6 doubles per point; wider superblocks need
    // fewer, and beyond the cap the one-sided kernel (at most 64 slots) is used instead
    for (;; w *= 2) {
        const int64_t S = (T + rows * w - 1) / (rows * w);
        const bool fits = (S + 1) * 6 * n * (int64_t)sizeof(double) <= kSymMaxPartBytes;
        if (fits && S * (S + 1) / 2 < ((int64_t)1 << 31)) {
            sp.waves = w;
            sp.rows = rows;
            sp.nsb = S;
            return sp;
        }
        if (w >= kSymMaxWaves || fixed) return sp;
    }
}

}  // namespace lm
