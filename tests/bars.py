"""Parity bars shared by the GPU tests.

FP64 path: 1e-9 relative per partition value (|F| floored at 1, the scale of
the noise-only statistic), plus FP64_KCOND * cond(M_l) for ill-conditioned
partitions.  Any two correct FP64 evaluations of 1/2 N^T M^{-1} N differ by
about eps * cond(M) relative (backward-stable solve; the noise component along
the weak eigen-direction is amplified by cond).  Measured against the
50-digit end-to-end reference (Sec. II.A, Eq. coherent_F_stat, on 64-bin
inputs): the oracle errs by at most 0.15 eps cond and the HIP FP64 path by at
most 0.375 eps cond; the HIP path against the oracle differs by at most
1.26 eps cond over 16,384 particles x 256 partitions of the 20,972-bin
workload.  The constant is 4 eps: three times the largest measured ratio.
"""
EPS = 2.0 ** -52
FP64_REL = 1e-9
FP64_KCOND = 4.0 * EPS
