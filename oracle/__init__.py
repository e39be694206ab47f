"""FP64 CPU oracle of the differentiable tile rasterizer (test infrastructure).

This package is the checker, not the product.  Only the test-suite, the smoke
entry and the CPU-baseline leg of the benchmark may import it; the HIP library
never links or calls it and shares no code, table or constant generator with
it.  It computes, plainly and slowly, in float64 numpy:

* ``camera``   pinhole intrinsics and the structured orbit of look-at views;
* ``sh``       real spherical harmonics up to degree 3 and their gradient;
* ``project``  EWA projection, culling, tile rectangles and SH colour;
* ``binning``  per-tile lists ordered by (tile, depth bits, index), keys, ranges;
* ``blend``    front-to-back compositing (per-pixel loop and per-tile form) and
               its exact derivative;
* ``loss``     (1 - lambda) L1 + lambda (1 - SSIM) and its image gradient;
* ``backward`` chain rule from screen-space gradients to the parameters;
* ``adam``     the bias-corrected Adam update;
* ``init``     Gaussians from isosurface points with a Philox4x32-10 stream;
* ``pipeline`` the whole per-view forward/backward built from the above;
* ``density``  adaptive density control (statistics, clone, split, prune,
               opacity reset);
* ``metrics``  image-quality metrics (MSE, PSNR, L1, SSIM) of a view.

The paper adopts the 3D-GS rasterizer by citation (Sec. III, Method Overview)
and states none of its formulas; each function names the reading it follows.
Where a reading has no independent pin in the test-suite the function says
"parity unpinned".
"""
