"""Oracle for the NUFFT dipole-dipole interaction (DDI) path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constants with the HIP library; both sides receive their inputs from
``paper_1504_02897_amd.inputs``, which holds no arithmetic of the method.

Contents
--------
``ddi_oracle``  plain FP64 evaluation of the spherical/polar Fourier quadrature
                of the DDI (Bao, Tang & Zhang, Sec. 2.1, Eqs. DDI-Con and
                DDI-Trun1) by direct nonuniform DFTs, its literal adjoint, the
                GPE energy split and gradient (Sec. 3.2), one gradient-flow
                step (Sec. 3.1, Eqs. gf-eq2, gf-colb2, gffg33), one time-splitting
                step (Sec. 4.1, Eq. tssp2) and the split I_1 + I_2 of Eq. 3.9
                (3D: the short-range part by the zero-padded FFT, the long-range
                part by direct sums over a small ball).
``refs``        analytic references used to pin the oracle: the 3D Gaussian
                closed form (Ex. 2.1, Eqs. extDensGausDipolar and Hessian_Ex1),
                the 2D Gaussian Bessel form (Ex. 2.2) and the 1D heat-kernel
                integrals for axis-aligned Gaussians (Ex. 2.3, Eqs.
                Coulomb:2D:aniso, Coulomb:3D:aniso:z, Coulomb:3D:aniso:xy).

Parity status of each function is stated in its docstring; every function is
pinned by a ``-m "not gpu"`` test except where it says "parity unpinned".
"""
