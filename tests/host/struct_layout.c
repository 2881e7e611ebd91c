/* Prints the size and field offsets of the public structs of cq.h, for the
 * check of the Python binding's ctypes mirrors. */
#include <stddef.h>
#include <stdio.h>

#include "cq.h"

#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))

int main(void)
{
    printf("cq_job size %zu\n", sizeof(cq_job));
    F(cq_job, img); F(cq_job, H); F(cq_job, W); F(cq_job, row_stride_bytes); F(cq_job, K);
    F(cq_job, scheme); F(cq_job, seed); F(cq_job, max_iters); F(cq_job, tol); F(cq_job, prune);
    F(cq_job, palette); F(cq_job, out_idx); F(cq_job, out_rgb); F(cq_job, subsample);
    printf("cq_stats size %zu\n", sizeof(cq_stats));
    printf("cq_engine_done size %zu\n", sizeof(cq_engine_done));
    F(cq_engine_done, ticket); F(cq_engine_done, status); F(cq_engine_done, stats);
    printf("cq_schedule size %zu\n", sizeof(cq_schedule));
    F(cq_schedule, min_colours); F(cq_schedule, assign_chunk); F(cq_schedule, regroup_period);
    return 0;
}
