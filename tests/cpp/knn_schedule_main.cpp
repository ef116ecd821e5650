// Walks the tile-pair schedules of the kNN kernels on the host: every ordered pair of tiles
// is met exactly once (row side, plus the column side under the symmetric schedule), the
// closed-form pair <-> index maps invert each other, and the incremental walks the kernels
// use agree with them.  Built by tests/test_knn_schedule.py from the helpers in knn.hip.
int main(int argc, char** argv) {
  const int64_t tmax = argc > 1 ? atoll(argv[1]) : 300;
  int bad = 0;
  for (int64_t T = 1; T <= tmax; ++T) {
    for (int sym = 0; sym <= 1; ++sym) {
      if (sym && T < 2) continue;
      const TileSched s = make_sched(T * KBQ - (T > 1 ? 5 : 0), sym);
      if (s.T != T) { printf("tile count T=%ld\n", (long)T); return 1; }
      std::vector<int> seen(T * T, 0);
      const int64_t P = a_pairs(s);
      std::vector<int> bseen(sym ? b_pairs(s) : 0, 0);
      int64_t i = 0, d = 0;
      for (int64_t t = 0; t < P; ++t) {
        int64_t i2, d2;
        a_pair(s, t, i2, d2);
        if (i2 != i || d2 != d) { printf("a_pair T=%ld t=%ld\n", (long)T, (long)t); ++bad; }
        if (t != a_start(s, i) + d || d >= a_len(s, i)) { printf("a_start/a_len T=%ld\n", (long)T); ++bad; }
        const int64_t j = a_db(s, i, d);
        seen[i * T + j]++;
        if (sym && j != i) seen[j * T + i]++;
        if (sym && d > 0) {
          const int64_t bi = b_index(s, i, d);
          if (bi < 0 || bi >= (int64_t)bseen.size()) { printf("b_index range T=%ld\n", (long)T); ++bad; continue; }
          bseen[bi]++;
          int64_t jj, dd;
          b_pair(s, bi, jj, dd);
          if (jj != j || dd != d || (jj - dd + T) % T != i) { printf("b_pair T=%ld\n", (long)T); ++bad; }
          if (bi != b_start(s, jj) + dd - 1 || dd > b_len(s, jj)) { printf("b_start/b_len T=%ld\n", (long)T); ++bad; }
        }
        a_next(s, i, d);
      }
      for (int64_t x = 0; x < T * T; ++x)
        if (seen[x] != 1) { printf("coverage T=%ld sym=%d pair %ld seen %d\n", (long)T, sym, (long)x, seen[x]); ++bad; break; }
      for (size_t x = 0; x < bseen.size(); ++x)
        if (bseen[x] != 1) { printf("column coverage T=%ld\n", (long)T); ++bad; break; }
      int64_t sum = 0;
      for (int64_t r = 0; r < T; ++r) { if (a_start(s, r) != sum) ++bad; sum += a_len(s, r); }
      if (sum != P) { printf("a_pairs T=%ld\n", (long)T); ++bad; }
      if (sym) {
        sum = 0;
        for (int64_t c = 0; c < T; ++c) { if (b_start(s, c) != sum) ++bad; sum += b_len(s, c); }
        if (sum != b_pairs(s)) { printf("b_pairs T=%ld\n", (long)T); ++bad; }
        int64_t j = 0, dd = 1;
        if (b_pairs(s) > 0) b_pair(s, 0, j, dd);
        for (int64_t t = 0; t < b_pairs(s); ++t) {   // the column kernel's incremental walk
          int64_t j2, d2;
          b_pair(s, t, j2, d2);
          if (j2 != j || d2 != dd) { printf("column walk T=%ld\n", (long)T); ++bad; break; }
          if (++dd > b_len(s, j)) { ++j; dd = 1; }
        }
      }
    }
  }
  printf("bad=%d\n", bad);
  return bad != 0;
}
