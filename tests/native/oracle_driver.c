/* Test driver: runs the oracle on instances read from stdin and prints the
 * deletion rounds, so that the oracle can be built and run under the
 * address and undefined-behaviour sanitizers.  Input: per instance a line
 * "n m mode" then m lines "f k v1 .. vk"; output: rounds, death_e, death_v. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int mhs_oracle_run(int32_t n, int32_t m, const int64_t *edge_ptr, const int32_t *edge_vtx,
                   const int32_t *demand, int mode, int32_t max_rounds, int32_t *death_e,
                   int32_t *death_v, int32_t *rounds);

int main(void) {
    int n, m, mode;
    while (scanf("%d %d %d", &n, &m, &mode) == 3) {
        int64_t *ptr = malloc(sizeof(int64_t) * (size_t)(m + 1));
        int32_t *dem = malloc(sizeof(int32_t) * (size_t)(m + 1));
        int cap = 16, nnz = 0;
        int32_t *vtx = malloc(sizeof(int32_t) * (size_t)cap);
        ptr[0] = 0;
        for (int e = 0; e < m; e++) {
            int f, k;
            if (scanf("%d %d", &f, &k) != 2) return 2;
            dem[e] = f;
            for (int i = 0; i < k; i++) {
                if (nnz == cap) { cap *= 2; vtx = realloc(vtx, sizeof(int32_t) * (size_t)cap); }
                if (scanf("%d", &vtx[nnz]) != 1) return 2;
                nnz++;
            }
            ptr[e + 1] = nnz;
        }
        int32_t *de = malloc(sizeof(int32_t) * (size_t)(m + 1));
        int32_t *dv = malloc(sizeof(int32_t) * (size_t)(n + 1));
        int32_t rounds = 0;
        int rc = mhs_oracle_run(n, m, ptr, vtx, dem, mode, -1, de, dv, &rounds);
        printf("%d %d\n", rc, rounds);
        for (int e = 0; e < m; e++) printf("%d ", de[e]);
        printf("\n");
        for (int v = 0; v < n; v++) printf("%d ", dv[v]);
        printf("\n");
        free(ptr); free(dem); free(vtx); free(de); free(dv);
    }
    return 0;
}
