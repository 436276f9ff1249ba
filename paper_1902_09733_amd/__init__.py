"""MI355X-native hierarchical belief-propagation stereo (libbpstereo bindings).

The stereo path of "Towards Real-time 3D Reconstruction using Consumer UAVs"
(Sec. 2.2): truncated absolute-difference cost volume, coarse-to-fine
checkerboard min-sum BP (Eq. 1), argmin/soft-argmin readout and joint
bilateral upsampling (Eq. 2), run by hand-written HIP kernels for gfx950
behind the C ABI in include/bp.h.
"""
from .stereo import (BPParams, Camera, Intrinsics, Pair, Workspace, backward, harris, icp, zssd_match, checkpoint_bytes, cost_volume, downsample,  # noqa: F401
                     run, run_noalloc, undistort, upsample, upsample_points, variant_count, workspace_bytes)
from .autograd import BPSoftArgmin, soft_argmin_bp  # noqa: F401
