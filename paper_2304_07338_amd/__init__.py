"""Photon Field Networks (arXiv 2304.07338) on MI355X: the photon-field ray-march hot path as
hand-written gfx950 HIP kernels behind the C ABI in include/pfn.h.

    from paper_2304_07338_amd.pfn import Context, RenderConfig, FieldConfig, TrainConfig
"""
from . import scenegen  # noqa: F401  (input generator; no method arithmetic)

__all__ = ["scenegen", "pfn", "workloads"]
