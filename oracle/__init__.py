"""CPU oracle for the multi-resolution screen-space lighting method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import anything from here.  The
product path (the HIP library and its Python binding) never imports, links or
calls this package, and this package never imports the product.

What it computes (Besenthal, Maisch, Ropinski, "Multi-Resolution Rendering
for Computationally Expensive Lighting Effects", arXiv 1906.04576):

* ``masks``   - Sec. 3.1: edge image from depth (second difference) and normal
                (first difference) discontinuities; downsample to every
                sub-image resolution; Gaussian blur with the Table 1
                variances; stencil = mask > 0 (Sec. 4.1); nested (inclusive)
                levels; owner-level partition and per-level work lists.
* ``ssao``    - Sec. 2.4 / 3.2 / 4.1: the occlusion estimator evaluated per
                sub-image only where its stencil permits, and the plain
                full-resolution pass used as the speed/quality reference
                (Sec. 5).
* ``merge``   - Sec. 3.3 / 4.2, Eq. 1: bilinear upsampling of every sub-image
                and the sequential blend from the coarsest level with
                alpha = min(a_i w_i, 1).
* ``shadow``  - Sec. 2.4 / 3.1: shadow-map hard test, shadow edges added to the
                mask, percentage-closer soft shadows.
* ``ssgi``    - Sec. 2.4: one-bounce screen-space indirect light.
* ``bilateral`` - Sec. 4.1: optional depth-aware blur of SSAO sub-images
                inside each level's stencil.
* ``frame_fullres_levels`` - Sec. 6: sub-images realised at full resolution
                with fewer samples, blended with the masks' alpha.
* ``frame``   - the whole per-frame pipeline for one effect.

Arithmetic contract (so the GPU path can be compared bit for bit): every
function takes ``dtype`` (np.float32 for parity, np.float64 for the error
twin); every written operation is one IEEE operation rounded to ``dtype``,
evaluated in the parenthesised order shown in the comments, with no fused
multiply-add and no reassociation.  numpy elementwise +, -, *, / and sqrt are
correctly rounded, floor/abs/min/max are exact.

Where the paper is silent the oracle takes one fixed reading; each such
reading is marked "reading:" at the place it is used.
"""
from .masks import (MaskParams, edge_image, foveate, gaussian_weights, blur_radius, or_pool,
                    build_pyramid, Pyramid, level_sample, work_lists, level_dims)
from .ssao import SSAOParams, ssao_texels, ssao_level, ssao_plain
from .merge import upsample_merge, upsampled_alpha
from .shadow import ShadowParams, light_coords, hard_shadow, shadow_edges, pcss_texels, pcss_level
from .ssgi import SSGIParams, ssgi_texels, ssgi_level
from .bilateral import BilateralParams, binomial_weights, bilateral_level
from .frame import frame, frame_fullres_levels, Frame

__all__ = [
    "MaskParams", "edge_image", "foveate", "gaussian_weights", "blur_radius", "or_pool", "build_pyramid",
    "Pyramid", "level_sample", "work_lists", "level_dims", "SSAOParams", "ssao_texels",
    "ssao_level", "ssao_plain", "upsample_merge", "ShadowParams", "light_coords", "hard_shadow",
    "shadow_edges", "pcss_texels", "pcss_level", "SSGIParams", "ssgi_texels", "ssgi_level",
    "BilateralParams", "binomial_weights", "bilateral_level", "frame", "frame_fullres_levels", "Frame",
    "upsampled_alpha",
]
