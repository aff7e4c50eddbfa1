// Instantiations of the vector training kernel with learned shading frames (Sec. 4.2; the
// frame layer trained with the decoder and the latents, Sec. 5).
#include "train_vec.h"

namespace nam {

bool train_frames_supported(const MlpShape& sh) {
    return (sh.NF == 1 || sh.NF == 2) && (sh.C == 8 || sh.C == 16) && (sh.H == 32 || sh.H == 64) &&
           (sh.NH == 2 || sh.NH == 3) && sh.NO == 3;
}

template <int MODE>
static hipError_t dispatch_frames(const MlpShape& sh, const TrainArgs& a, int grid, hipStream_t s) {
#define NAM_TF_CASE(C_, H_, NH_, NF_)                                                       \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_ && sh.NF == NF_) {                        \
        clear_stale_hip_error();                                                            \
        fwdbwd_kernel<C_, H_, NH_, 3, MODE, NF_><<<grid, kTW, 0, s>>>(a);                  \
        return hipGetLastError();                                                           \
    }
#define NAM_TF_NF(C_, H_, NH_) NAM_TF_CASE(C_, H_, NH_, 1) NAM_TF_CASE(C_, H_, NH_, 2)
    NAM_TF_NF(8, 32, 2) NAM_TF_NF(8, 32, 3) NAM_TF_NF(8, 64, 2) NAM_TF_NF(8, 64, 3)
    NAM_TF_NF(16, 32, 2) NAM_TF_NF(16, 32, 3) NAM_TF_NF(16, 64, 2) NAM_TF_NF(16, 64, 3)
#undef NAM_TF_NF
#undef NAM_TF_CASE
    return hipErrorInvalidValue;
}

template <int MODE>
static int occupancy_frames(const MlpShape& sh) {
    int b = 0;
#define NAM_TF_O(C_, H_, NH_, NF_)                                                          \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_ && sh.NF == NF_)                          \
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)fwdbwd_kernel<C_, H_, NH_, 3, MODE, NF_>, kTW, 0);
#define NAM_TF_ONF(C_, H_, NH_) NAM_TF_O(C_, H_, NH_, 1) NAM_TF_O(C_, H_, NH_, 2)
    NAM_TF_ONF(8, 32, 2) NAM_TF_ONF(8, 32, 3) NAM_TF_ONF(8, 64, 2) NAM_TF_ONF(8, 64, 3)
    NAM_TF_ONF(16, 32, 2) NAM_TF_ONF(16, 32, 3) NAM_TF_ONF(16, 64, 2) NAM_TF_ONF(16, 64, 3)
#undef NAM_TF_ONF
#undef NAM_TF_O
    return b < 1 ? 1 : b;
}

hipError_t launch_fwdbwd_frames(const MlpShape& sh, int mode, const TrainArgs& a, int grid, hipStream_t s) {
    if (mode == kModeForward) return dispatch_frames<kModeForward>(sh, a, grid, s);
    if (mode == kModeLoss) return dispatch_frames<kModeLoss>(sh, a, grid, s);
    return dispatch_frames<kModeGrad>(sh, a, grid, s);
}

int fwdbwd_frames_blocks_per_cu(const MlpShape& sh, int mode) {
    if (mode == kModeForward) return occupancy_frames<kModeForward>(sh);
    if (mode == kModeLoss) return occupancy_frames<kModeLoss>(sh);
    return occupancy_frames<kModeGrad>(sh);
}

}  // namespace nam
