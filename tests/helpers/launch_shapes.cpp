// Prints the host-side launch shapes of the Metropolis colour kernels and the
// Swendsen-Wang tile counts for every L read from stdin, one line per L:
// L quad rows row_blocks tiles
#include <stdio.h>

#include "cvf_internal.h"
#include "met_launch.h"

int main()
{
    unsigned L;
    while (scanf("%u", &L) == 1) {
        const cvf::MetShape m = cvf::met_shape(L);
        printf("%u %u %u %u %zu\n", L, m.quad, m.rows, m.row_blocks, cvf::sw_tiles_of(L));
    }
    return 0;
}
