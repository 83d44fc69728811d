// Instantiates the EM kernels for D = 3 with double iterations.
#include "gm_compress_impl.h"

namespace gm {

int launch_compress_d3_double(int kmax_tpl, int per_thread, int mode, int waves, const CompressArgs& a, int grid,
                          hipStream_t st)
{
    return launch_bucket_dr<3, double>(kmax_tpl, per_thread, mode, waves, a, grid, st);
}

int grid_compress_d3_double(int kmax_tpl, int per_thread, int mode, int waves)
{
    return grid_dr<3, double>(kmax_tpl, per_thread, mode, waves);
}


int launch_compress_big_d3_double(int kmax_tpl, const CompressArgs& a, int grid, hipStream_t st)
{
    return launch_big_dr<3, double>(kmax_tpl, a, grid, st);
}

}  // namespace gm
