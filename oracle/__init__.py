"""CPU float64 oracle for spatially adaptive (extended) correlation and convolution.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously correct reference
that the HIP path is checked against. Only the tests, the smoke check and the
bench's CPU-baseline leg may import it; the product path never does, and it shares
no code, tables or helpers with the HIP library.

Everything here follows "Efficient Spatially Adaptive Convolution and Correlation"
(arXiv 2006.13188):
  * definitions of extended correlation / convolution: Sec. 2.1 eq. (Def-ECorr),
    Sec. 2.2 eq. (Def-EConv);
  * the rotation algorithm: Sec. 4.1 (filter decomposition, standard correlations,
    linear combination, and the pre-multiplied convolution);
  * band-limiting: Sec. 4.3;
  * scale group and normalisation: Sec. 8, eq. (normalization), normalised signal;
  * normalised filtering with a rotation field (line-integral convolution): Sec. 8;
  * pattern detection (gradient signal and field, consensus filter by voting, peaks): Sec. 5;
  * joint rotation and scale fields (the Conclusion's future work): joint.py;
  * steering in 3D (spherical harmonics per radius, Wigner-D combination): Sec. 9,
    steer3d.py.

Readings where the paper is silent are listed per function (boundary = zero outside
the image, bilinear polar resampling at the exact grid radii, k = -K..K, etc.).

Parity status: every function below is pinned by tests in tests/test_oracle_*.py
except the scale-group coefficients c_k and the joint coefficients c_{k,l}, whose values
are fixed only by the readings of those decompositions (parity unpinned; see scale.py and
joint.py).
"""
from .decompose import (
    default_angular_samples, bilinear, grid_radii, angular_components,
    rotated_filter, half_components,
)
from .extended import (
    ext_corr_brute, ext_conv_brute, ext_corr_fft, ext_conv_fft,
    ext_conv_half, ext_corr_half, match_rotations, min_fft_size, fft_workers,
)
from .adjoint import conv_backward, corr_backward
from .normalized import normalized_conv_brute, normalized_conv_fft, normalized_conv_half
from .detection import gradient_field, voting_filter, find_peaks, detection_response
from .joint import JointParams, joint_components, joint_filter_at, joint_conv_brute, joint_conv_fft, joint_smooth
from .steer3d import (
    sh_coefficients, half_set, components3d, euler_matrix, wigner_small_d, wigner_D,
    ext_corr3d_brute, ext_conv3d_brute, ext_corr3d_fft, ext_conv3d_fft,
)
from .scale import (
    ScaleParams, scale_components, scale_filter_at, scale_smooth_brute,
    scale_smooth_fft,
)

__all__ = [
    "default_angular_samples", "bilinear", "grid_radii", "angular_components",
    "rotated_filter", "half_components",
    "ext_corr_brute", "ext_conv_brute", "ext_corr_fft", "ext_conv_fft",
    "ext_conv_half", "ext_corr_half", "match_rotations", "min_fft_size", "fft_workers",
    "conv_backward", "corr_backward",
    "normalized_conv_brute", "normalized_conv_fft", "normalized_conv_half",
    "gradient_field", "voting_filter", "find_peaks", "detection_response",
    "JointParams", "joint_components", "joint_filter_at", "joint_conv_brute", "joint_conv_fft", "joint_smooth",
    "ScaleParams", "scale_components", "scale_filter_at", "scale_smooth_brute",
    "scale_smooth_fft",
    "sh_coefficients", "half_set", "components3d", "euler_matrix", "wigner_small_d", "wigner_D",
    "ext_corr3d_brute", "ext_conv3d_brute", "ext_corr3d_fft", "ext_conv3d_fft",
]
