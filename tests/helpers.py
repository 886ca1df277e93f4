"""Error metrics shared by the parity tests."""
import numpy as np


def per_scale_rel_l2(got, ref, floor=1e-3):
    """e_j = ||got_j - ref_j||_2 / max(||ref_j||_2, floor * max_k ||ref_k||_2)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    nrm = np.linalg.norm(ref, axis=-1)
    den = np.maximum(nrm, floor * nrm.max())
    return np.linalg.norm(got - ref, axis=-1) / den


def error_spectrum_percent(got, ref):
    """ES of Sec. 4.1 (Eq. error_spectrum): per-scale L1 error relative to the
    reference, in percent."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    return 100.0 * np.sum(np.abs(got - ref), axis=-1) / np.sum(np.abs(ref), axis=-1)
