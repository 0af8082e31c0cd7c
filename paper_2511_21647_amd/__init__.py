"""MI355X-native projection-based RCA ULM reconstruction.

The hot path (two-stage beamforming to projection planes, eigen-based SVD
clutter filter, NCC or CNN localisation) runs in libulmproj.so's HIP kernels;
this package only marshals arguments to its C ABI.
"""
from ._lib import (ULM_OK, ULM_ERR_INVALID_ARG, ULM_ERR_HIP, ULM_ERR_OVERFLOW, ULM_ERR_NUMERIC,
                   ULM_ERR_NOT_IMPLEMENTED, LOC3D_DTYPE, ulm_stage1_slices,
                   ulm_motion_workspace_size, ulm_motion_estimate, ulm_separate, loc3d_to_numpy, ulm_pair_planes, ulm_pair_workspace_size,
                   ulm_pair_planes_noalloc, ULM_NOALLOC_SCRATCH_BYTES,
                   CNN_LAYOUT, CNN_THRESHOLD, CNN_UPSAMPLE, ULM_CNN_BF16, ULM_CNN_FP32, ULM_CNN_PARAMS, Workspace,
                   cnn_pack, cnn_unpack, ulm_cnn_forward, ulm_cnn_gradients, ulm_cnn_images,
                   ulm_cnn_localize, ulm_cnn_localize_workspace_size, ulm_cnn_train_step,
                   ulm_cnn_workspace_size,
                   LOC_DTYPE, ULM_PREC_BF16X3, ULM_PREC_FP64GRAM, Context, ULMConfig, ULMError,
                   locs_to_numpy, make_config, ncc_localize, rca_beamform_proj, rca_beamform_stage1,
                   rca_beamform_stage2, rca_beamform_cross, ulm_xdoppler, svd_clutter_filter,
                   ulm_check_status, ulm_density_accumulate, ulm_reconstruct_ensemble,
                   ulm_reconstruct_ensemble_cnn,
                   ulm_sim_channel_data, LIB_PATH)

__all__ = ["ULM_OK", "ULM_ERR_INVALID_ARG", "ULM_ERR_HIP", "ULM_ERR_OVERFLOW", "ULM_ERR_NUMERIC",
           "ULM_ERR_NOT_IMPLEMENTED", "LOC3D_DTYPE", "ulm_stage1_slices",
           "ulm_motion_workspace_size", "ulm_motion_estimate", "ulm_separate", "loc3d_to_numpy", "ulm_pair_planes", "ulm_pair_workspace_size",
           "ulm_pair_planes_noalloc", "ULM_NOALLOC_SCRATCH_BYTES",
           "LOC_DTYPE", "ULM_PREC_BF16X3", "ULM_PREC_FP64GRAM", "Context", "ULMConfig",
           "ULMError", "locs_to_numpy", "make_config", "ncc_localize", "rca_beamform_proj", "rca_beamform_stage1", "rca_beamform_stage2",
           "rca_beamform_cross", "ulm_xdoppler",
           "svd_clutter_filter", "ulm_check_status", "ulm_density_accumulate",
           "ulm_reconstruct_ensemble", "ulm_reconstruct_ensemble_cnn", "ulm_sim_channel_data", "LIB_PATH",
           "CNN_LAYOUT", "CNN_THRESHOLD", "CNN_UPSAMPLE", "ULM_CNN_BF16", "ULM_CNN_FP32", "ULM_CNN_PARAMS",
           "Workspace", "cnn_pack", "cnn_unpack", "ulm_cnn_forward", "ulm_cnn_gradients",
           "ulm_cnn_images", "ulm_cnn_localize", "ulm_cnn_localize_workspace_size",
           "ulm_cnn_train_step", "ulm_cnn_workspace_size"]
