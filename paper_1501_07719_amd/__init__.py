"""MI355X RIME chi-squared engine: Python binding of librime.so.

``rime`` holds the ctypes binding of the C ABI (include/rime.h) and
``autograd`` a torch.autograd.Function over the fused chi^2 + adjoint.
"""
from .rime import (  # noqa: F401
    FP64, MIXED, MIXED_RES64, MODE_CHI2, MODE_CHI2_GRAD, MODE_PREDICT, RIME_ERR_DOMAIN, Batch,
    DeviceSky, Plan, RimeError, load_library, rime_autotune, rime_batch_autotune,
    rime_batch_create, rime_batch_get_variant, rime_batch_set_variant, rime_chi2,
    rime_chi2_batched, rime_chi2_ex, rime_chi2_grad, rime_chi2_grad_noalloc, rime_chi2_streamed, rime_domain_status,
    rime_loglike_const, rime_predict, rime_predict_ex, rime_streamed_workspace_size,
    rime_tiling_host, rime_variant_count, rime_variant_info, rime_variant_matrix_cores,
    rime_workspace_size, rime_workspace_size_ex, workspace,
)
