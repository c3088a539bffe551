/* nlo_duffy.c - oracle for vertex-sharing element pairs under the singular
 * (fractional) kernel.  TEST INFRASTRUCTURE ONLY.  Filled in below. */
#include "nlo.h"
int nlo_duffy_block(const nlo_mesh *m, const nlo_problem *p, int k, int kp, double blk[36])
{
    (void)m; (void)p; (void)k; (void)kp; (void)blk;
    return -3;
}
