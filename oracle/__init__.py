"""FP64 CPU oracle for the differentiable C-ToF Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP implementation.

Modules
-------
binning    -- per (frame, Gaussian) projection, tile rectangle and depth key in
              FP64 with a fixed operation order (numpy), and the sorted
              (frame, tile, depth key, index) pair lists.
render     -- the image formation model of paper §3 (Eq. 2 RGB, Eq. 4 raw
              quads, Eq. 5 mean depth) evaluated per pixel in exact sorted
              order, in FP64 (torch CPU tensors), with gradients by autograd.
recursion  -- the per-pixel opacity-gradient recursion of the supplement
              (Eqs. S2, S3) plus the background term, in numpy FP64.
brute      -- per-pixel double loop in plain Python floats for tiny scenes.
optim      -- L2 loss and Adam (paper §4 hyperparameters) in FP64.
sh         -- real spherical harmonics up to degree 3 (view-dependent colour).
tof        -- the time-of-flight epilogue: phasor, d_ToF and amplitude.
mlp        -- the deformation network of §4: positional encoding, MLP,
              per-(time, Gaussian) centre offsets and their gradients.

Parity status: every function here is pinned by tests in tests/ against
closed forms, brute force or finite differences; see each module header.
"""
