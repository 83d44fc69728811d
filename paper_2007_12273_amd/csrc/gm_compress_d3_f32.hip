// Instantiates the EM kernels for D = 3 with float iterations.
#include "gm_compress_impl.h"

namespace gm {

int launch_compress_d3_float(int kmax_tpl, int per_thread, int mode, int waves, const CompressArgs& a, int grid,
                          hipStream_t st)
{
    return launch_bucket_dr<3, float>(kmax_tpl, per_thread, mode, waves, a, grid, st);
}

int grid_compress_d3_float(int kmax_tpl, int per_thread, int mode, int waves)
{
    return grid_dr<3, float>(kmax_tpl, per_thread, mode, waves);
}

int launch_compress_pre_d3(const CompressArgs& a, hipStream_t st) { return launch_pre_dr<3>(a, st); }

int launch_compress_requeue_d3(const CompressArgs& a, hipStream_t st) { return launch_requeue_dr<3>(a, st); }

int launch_compress_finish_d3(int kmax_tpl, const CompressArgs& a, hipStream_t st)
{
    return launch_finish_dr<3>(kmax_tpl, a, st);
}


int launch_compress_big_d3_float(int kmax_tpl, const CompressArgs& a, int grid, hipStream_t st)
{
    return launch_big_dr<3, float>(kmax_tpl, a, grid, st);
}

}  // namespace gm
