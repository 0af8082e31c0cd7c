"""MI355X-native projection-based RCA ULM reconstruction.

The hot path (two-stage beamforming to projection planes, eigen-based SVD
clutter filter, NCC localisation) runs in libulmproj.so's HIP kernels; this
package only marshals arguments to its C ABI.
"""
from ._lib import (LOC_DTYPE, ULM_PREC_BF16X3, ULM_PREC_FP64GRAM, Context, ULMConfig, ULMError,
                   locs_to_numpy, make_config, ncc_localize, rca_beamform_proj, rca_beamform_stage1,
                   rca_beamform_stage2, svd_clutter_filter,
                   ulm_check_status, ulm_density_accumulate, ulm_reconstruct_ensemble,
                   ulm_sim_channel_data, LIB_PATH)

__all__ = ["LOC_DTYPE", "ULM_PREC_BF16X3", "ULM_PREC_FP64GRAM", "Context", "ULMConfig",
           "ULMError", "locs_to_numpy", "make_config", "ncc_localize", "rca_beamform_proj", "rca_beamform_stage1", "rca_beamform_stage2",
           "svd_clutter_filter", "ulm_check_status", "ulm_density_accumulate",
           "ulm_reconstruct_ensemble", "ulm_sim_channel_data", "LIB_PATH"]
