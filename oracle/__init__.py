"""FP64 CPU oracle for the 2D-Gaussian frame-fitting path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, helpers or tables) and imports nothing from it.

What it computes, each function citing the passage it follows:

* ``render``   - Eq. 2 (accumulated summation, Sec. 3.1) evaluated as a plain
                 per-pixel sum over all Gaussians (brute force) and over each
                 Gaussian's 3-sigma box; the covariance is Eq. 1 (Sigma = L L^T)
                 used in its conic (inverse-covariance) form.
* ``binning``  - the tile lists a tile-based rasteriser needs (Sec. 3, the
                 tile-based differentiable rasterisation the method inherits),
                 specified in FP32 with a fixed operation order.
* ``loss``     - mean-squared error, its gradient and PSNR.
* ``grads``    - analytic gradients of the loss w.r.t. every Gaussian
                 parameter (mu, Cholesky vector l, colour c') by the chain
                 rule through the conic form.
* ``fd``       - central finite differences of the brute-force loss.
* ``adam``     - the per-step parameter update of the fitting loop ("encoding
                 optimization steps", Sec. 4.1) taken as Adam.
* ``init``     - the content-aware ROI initialisation (Sec. 3.2.A), in the
                 gradient-magnitude-sampling form used for synthetic frames.
* ``fit``      - the loop render -> loss -> gradients -> Adam.
* ``quant``    - post-training quantisation of a fitted frame (binary16 means,
                 uniform min-max Cholesky and colour codes), its entropy-coded
                 bits and the bits-back saving of P-frames (Sec. 3.3, Eq. 3, 4).
* ``select``   - the P-frame change mask and the reference Gaussians that
                 influence a changed pixel (selective optimisation,
                 Sec. 3.2.C), specified in FP32.
* ``superpixel`` - the superpixel ROI initialisation (Sec. 3.2.A, Fig. 2):
                 SLIC-style K-means in (x, y, colour) from the content-aware
                 seeds, exact integer segment moments, one Gaussian per
                 segment from its centre, covariance and mean colour.

Every function works in float64 unless it states otherwise; binning, the
P-frame selection, the quantiser codes and the superpixel assignment are the
deliberate FP32 parts
because a tile list, a selected set and a code are integer decisions that
both sides must take in the same precision.
"""
