/* Sanitizer driver for the oracle (test infrastructure): built with
 * -fsanitize=address,undefined and run by tests/test_sanitizers.py.
 *
 * Each argument is a case file: a first line "G W lo hi seed0 n_seeds",
 * then the program text.  Every global array and scalar is bound to the
 * seeded range [lo, hi).  For every seed the driver prints one line
 * "<case> <seed> <status> <records> <race cells> <benign cells> <accesses>",
 * and for a text the parser rejects, "<case> parse-error". */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static char* slurp(const char* path) {
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  char* buf = (char*)malloc((size_t)n + 1);
  if (fread(buf, 1, (size_t)n, f) != (size_t)n) { fclose(f); free(buf); return NULL; }
  buf[n] = 0;
  fclose(f);
  return buf;
}

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    char* text = slurp(argv[a]);
    if (!text) { fprintf(stderr, "cannot read %s\n", argv[a]); return 2; }
    unsigned G, W, n;
    long long lo, hi;
    unsigned long long seed0;
    char* nl = strchr(text, '\n');
    if (!nl || sscanf(text, "%u %u %lld %lld %llu %u", &G, &W, &lo, &hi, &seed0, &n) != 6) {
      fprintf(stderr, "bad header in %s\n", argv[a]);
      return 2;
    }
    char err[256];
    orc_prog* p = orc_parse(nl + 1, err, sizeof err);
    if (!p) {
      printf("%s parse-error\n", argv[a]);
      free(text);
      continue;
    }
    const int na = orc_n_global_arrays(p), ns = orc_n_scalars(p);
    orc_bind arrays[16], scalars[16];
    for (int i = 0; i < na && i < 16; ++i) { memset(&arrays[i], 0, sizeof arrays[i]); arrays[i].lo = lo; arrays[i].hi = hi; }
    for (int i = 0; i < ns && i < 16; ++i) { memset(&scalars[i], 0, sizeof scalars[i]); scalars[i].lo = lo; scalars[i].hi = hi; }
    for (unsigned j = 0; j < n; ++j) {
      orc_result r;
      memset(&r, 0, sizeof r);
      if (orc_run(p, G, W, arrays, na, scalars, ns, seed0 + j, j, 0, -1, &r, err, sizeof err) != 0) {
        printf("%s %llu run-error %s\n", argv[a], seed0 + j, err);
        continue;
      }
      printf("%s %llu %d %llu %u %u %llu\n", argv[a], seed0 + j, r.summary.status,
             (unsigned long long)r.n_records, r.summary.n_race_cells, r.summary.n_benign_cells,
             (unsigned long long)r.summary.n_accesses);
      orc_result_free(&r);
    }
    orc_prog_free(p);
    free(text);
  }
  return 0;
}
