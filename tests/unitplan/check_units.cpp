// Checks the factor's unit plan (nnls_internal.h) on the host: for every block count nb,
// kept-column count j0 and strip shape, the units cover each computed tile exactly once,
// and every unit waits only for tiles that units with smaller tickets produce, the walker's
// outputs counting at the ticket of the last unit the walker needs for that column.
// Prints "ok <cases>" or the first violation.
#include <cstdio>
#include <map>
#include <utility>
#include <vector>

#include "nnls_internal.h"

using namespace nnls;

// kept_single: the kept columns' units are one-column strips that stop TD terms short and
// hand over partial tiles; the row walker of tile row I finishes (I, J) once the units of
// (I, 0 .. J) are through (it runs from the start of the launch on tickets of its own).
static int check(int nb, int j0, int RS, int RP, bool pairs, bool kept_single = false) {
  const UnitPlan p = {nb, j0, RS, RP, pairs, kept_single};
  constexpr int TD = WalkTD<float>::value;
  const int64_t total = unit_total(p);
  std::map<std::pair<int, int>, int64_t> producer;   // tile -> unit (the partial unit for walker tiles)
  std::vector<FactorUnit> units;
  for (int64_t t = 0; t < total; ++t) {
    const FactorUnit f = unit_at(t, p);
    units.push_back(f);
    const int C = f.kind == UNIT_PAIR ? 2 : 1;
    if (f.cnt < 1 || (f.kind == UNIT_TILE && f.cnt != 1)) return std::printf("bad cnt nb=%d j0=%d t=%lld\n", nb, j0, (long long)t), 1;
    for (int c = 0; c < C; ++c)
      for (int r = 0; r < f.cnt; ++r) {
        const int I = f.I + r, J = f.J + c;
        if (J >= nb || I >= nb || I < J || I < j0)
          return std::printf("tile (%d,%d) outside nb=%d j0=%d\n", I, J, nb, j0), 1;
        if (!producer.emplace(std::make_pair(I, J), t).second)
          return std::printf("tile (%d,%d) twice nb=%d j0=%d\n", I, J, nb, j0), 1;
        // strips hold plain off-diagonal tiles only (not the walker's inputs)
        if (f.kind != UNIT_TILE && J >= j0 && I - J <= 1)
          return std::printf("walker tile (%d,%d) in a strip nb=%d j0=%d\n", I, J, nb, j0), 1;
        if (kept_single && J < j0 && f.kind != UNIT_STRIP)
          return std::printf("kept tile (%d,%d) not in a one-column strip nb=%d j0=%d\n", I, J, nb, j0), 1;
      }
  }
  int64_t want = 0;
  for (int J = 0; J < nb; ++J) want += nb - (J > j0 ? J : j0);
  if ((int64_t)producer.size() != want) return std::printf("coverage %zu != %lld\n", producer.size(), (long long)want), 1;
  // the walker finishes column J (its diagonal inverse, and the final (J,J), (J+1,J)) once
  // the partial units of (J,J) and (J+1,J) and every earlier column are through
  std::vector<int64_t> walker(nb, -1);
  for (int J = j0; J < nb; ++J) {
    int64_t w = J > j0 ? walker[J - 1] : -1;
    w = std::max(w, producer.at({J, J}));
    if (J + 1 < nb) w = std::max(w, producer.at({J + 1, J}));
    walker[J] = w;
  }
  std::map<std::pair<int, int>, int64_t> rowdone;   // kept_single: the row walkers' finished tiles
  if (kept_single)
    for (int I = j0; I < nb; ++I) {
      int64_t w = -1;
      for (int J = 0; J < j0; ++J) rowdone[{I, J}] = w = std::max(w, producer.at({I, J}));
    }
  auto ready_at = [&](int I, int K) -> int64_t {   // ticket after which tile (I, K) is final
    if (I < j0 && K < j0) return -1;                // kept from the previous launch
    if (kept_single && K < j0) return rowdone.at({I, K});
    if (K >= j0 && I - K <= 1) return walker[K];    // the walker's diagonal and sub-diagonal
    return producer.at({I, K});
  };
  auto dinv_at = [&](int J) -> int64_t { return J < j0 ? -1 : walker[J]; };
  for (int64_t t = 0; t < total; ++t) {
    const FactorUnit& f = units[(size_t)t];
    const int C = f.kind == UNIT_PAIR ? 2 : 1;
    auto need = [&](int64_t at, const char* what) {
      if (at >= t) {
        std::printf("unit %lld (kind %d, I %d, J %d) waits for %s at %lld; nb=%d j0=%d\n", (long long)t, f.kind, f.I,
                    f.J, what, (long long)at, nb, j0);
        return false;
      }
      return true;
    };
    for (int c = 0; c < C; ++c)
      for (int r = 0; r < f.cnt; ++r) {
        const int I = f.I + r, J = f.J + c;
        const bool partial = (f.kind == UNIT_TILE && J >= j0 && I - J <= 1) || (kept_single && J < j0);
        int kend = (f.kind == UNIT_TILE && I == J && J > j0) ? J - 1 : (C == 2 ? f.J : J);
        if (kept_single && J < j0) kend = std::max(J - TD, 0);
        for (int k = 0; k < kend; ++k) {
          if (!need(ready_at(I, k), "L_Ik")) return 1;
          if (!need(ready_at(J, k), "L_Jk")) return 1;
        }
        if (c == 1) {   // a pair's second column: L_{J,J-1}; L_{I,J-1} is its own output
          if (!need(ready_at(J, J - 1), "L_{J,J-1}")) return 1;
        }
        if (!partial && !need(dinv_at(J), "L_JJ^-1")) return 1;
      }
  }
  return 0;
}

int main() {
  int cases = 0;
  for (int nb = 1; nb <= 40; ++nb)
    for (int j0 = 0; j0 < nb; ++j0)
      for (int shape = 0; shape < 4; ++shape) {
        const int RS = shape == 0 ? 1 : (shape == 1 ? 4 : (shape == 2 ? 2 : 3));
        const int RP = shape == 0 ? 1 : (shape == 1 ? 3 : (shape == 2 ? 1 : 2));
        const bool pairs = shape != 0;
        if (check(nb, j0, RS, RP, pairs)) return 1;
        ++cases;
        if (pairs && j0 > 0) {   // with row walkers for the rows below the kept block
          if (check(nb, j0, RS, RP, pairs, true)) return 1;
          ++cases;
        }
      }
  if (check(469, 0, CHOL_STRIP, CHOL_PAIR, true) || check(782, 613, CHOL_STRIP, CHOL_PAIR, true) ||
      check(199, 185, CHOL_STRIP, CHOL_PAIR, true, true) || check(196, 195, CHOL_STRIP, CHOL_PAIR, true, true))
    return 1;
  std::printf("ok %d\n", cases + 4);
  return 0;
}
