/* Brute-force density of states of the q-state Potts model on an L x L
 * periodic square lattice (Eq. 1): visits all q^(L*L) configurations and
 * counts them by (number of satisfied bonds, N_max).  Independent of the
 * oracle: shares no code with it.  Usage: enum_dos L q ; prints "E nmax count". */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  const int L = atoi(argv[1]), q = atoi(argv[2]), N = L * L;
  if (L < 2 || L > 5 || q < 2 || q > 4) return 2;
  uint64_t total = 1;
  for (int i = 0; i < N; ++i) total *= (uint64_t)q;
  const int EMAX = 2 * N;
  uint64_t *count = calloc((size_t)(EMAX + 1) * (size_t)(N + 1), sizeof(uint64_t));
  int *s = calloc((size_t)N, sizeof(int));
  if (!count || !s) return 3;
  for (uint64_t c = 0; c < total; ++c) {
    /* decode c in base q into the lattice, site 0 = least significant digit */
    uint64_t r = c;
    for (int i = 0; i < N; ++i) { s[i] = (int)(r % (uint64_t)q); r /= (uint64_t)q; }
    int e = 0;
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        const int v = s[y * L + x];
        e += (v == s[y * L + (x + 1) % L]);
        e += (v == s[((y + 1) % L) * L + x]);
      }
    int n[8] = {0};
    for (int i = 0; i < N; ++i) n[s[i]]++;
    int nmax = 0;
    for (int v = 0; v < q; ++v) if (n[v] > nmax) nmax = n[v];
    count[(size_t)e * (N + 1) + nmax]++;
  }
  for (int e = 0; e <= EMAX; ++e)
    for (int m = 0; m <= N; ++m)
      if (count[(size_t)e * (N + 1) + m]) printf("%d %d %llu\n", e, m, (unsigned long long)count[(size_t)e * (N + 1) + m]);
  free(count); free(s);
  return 0;
}
