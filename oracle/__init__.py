"""FP64 CPU oracle for the glint P-NDF range-query path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this package.  The GPU library
never calls it, and it shares no code with the GPU library: both sides are
written independently from the paper (Deng et al., "Constant-Cost
Spatio-Angular Prefiltering of Glinty Appearance Using Tensor
Decomposition").

Modules
-------
ndf     per-texel bin masses of the intrinsic-roughness Gaussian (Sec. 3.1,
        Eq. geom), the brute-force NDF tensor over every texel position and
        footprint level (Sec. 4.1), and the brute-force range integral.
cluster the paper's clustered layout (Sec. 4.2 practical choices): per
        region-and-angular-block 3-way CP-ALS and the block-split range query.
cp_als  plain CP decomposition by alternating least squares (Sec. 4.2,
        Eq. compress) and the texel-space MTTKRP identity used as a pin at
        sizes where the tensor cannot be formed.
query   summed-area (cumulative) tables (Sec. 4.4), point query (Sec. 4.3,
        Eq. decompress), range query (Sec. 4.4, Eq. rangeDecom and the
        Appendix proposition), its gradient, and the query conditioning
        magnitude used by the tolerances.
sampling  hierarchical NDF importance sampling by range queries (Sec. 5.2).
sg      environment-light prefiltering (Sec. 5.4): the compact-eps support of
        a spherical-Gaussian lobe as an angular box, averaged by range query.
wang    constant-storage synthesis with Wang tiles (Sec. 5.5): hashed edge
        colours, per-tile tensors with margins, sums over overlapped tiles.
quant   BF16 and FP8 (OCP E4M3FN) rounding with per-column scales.
adam    one Adam step (refinement of the factors; not in the paper).

Every function is plain and unfused; readings taken where the paper is silent
are listed in each module's docstring.
"""
