"""MI355X-native sparse-coefficient Gaussian splatting (LangSplatV2 hot path).

The HIP library ``libls2.so`` (C ABI in ``include/ls2.h``) does all the work;
this package marshals torch tensors into it.  Importing fails if the library
has not been built (there is no fallback path).
"""
from ._lib import (  # noqa: F401
    LS2_BF16,
    LS2_ERR_ARG,
    LS2_ERR_CAPACITY,
    LS2_ERR_DEVICE,
    LS2_ERR_UNSUPPORTED,
    LS2_F32,
    LS2_OK,
    LS2_SELECT_MASK_MEAN,
    LS2_SELECT_MAX,
    LS2_SMOOTH_AVG,
    LS2_SMOOTH_HALF,
    LS2Error,
    LIB_PATH,
    ls2_accumulate,
    ls2_bin_sort,
    ls2_bin_sort_count,
    ls2_bin_sort_workspace,
    ls2_decode_feature_loss,
    ls2_decode_feature_loss_workspace,
    ls2_dict_decode,
    ls2_dict_decode_backward,
    ls2_dict_decode_backward_workspace,
    ls2_feature_loss,
    ls2_feature_loss_workspace,
    ls2_postprocess,
    ls2_postprocess_workspace,
    ls2_project,
    ls2_project_backward,
    ls2_query,
    ls2_query_coef,
    ls2_query_coef_workspace,
    ls2_query_backward,
    ls2_sparse_codes,
    ls2_sparse_codes_backward,
    ls2_splat_dense,
    ls2_splat_sparse,
    ls2_splat_sparse_backward,
    make_camera,
    status_string,
    version,
)
from .render import Gradients, LS2Render, Pipeline, Trainer, to_device  # noqa: F401
