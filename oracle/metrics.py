"""Error and fidelity statistics between a reference amplitude set ``a`` and a
tested set ``b`` (oracle side; test infrastructure).

The paper states no precision and no error metric.  The readings used:

* rel_l2    = ||b - a||_2 / ||a||_2 over the batch (the gated quantity);
* max_scaled = max_i |b_i - a_i| / rms(a) (gated at 10x the tolerance);
* f_xeb     = (mean(2^N p_i * 2^N q_i) - 1) / (mean((2^N p_i)^2) - 1), with p
  the reference and q the tested probabilities (a cross-entropy style fidelity
  estimate; statistically noisy at small batch sizes, reported, not gated);
* f_ovl     = |sum conj(a) b|^2 / (sum |a|^2 sum |b|^2).

A per-amplitude relative error is ill-conditioned for near-zero amplitudes
(Porter-Thomas statistics), so it is reported as median and p99 only.
"""

import numpy as np


def compare(a: np.ndarray, b: np.ndarray, n_qubits: int) -> dict:
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    diff = np.abs(b - a)
    na = np.linalg.norm(a)
    rms = na / np.sqrt(max(a.size, 1))
    rel = diff / np.maximum(np.abs(a), 1e-300)
    p = np.abs(a) ** 2 * 2.0 ** n_qubits
    q = np.abs(b) ** 2 * 2.0 ** n_qubits
    den = np.mean(p * p) - 1.0
    f_xeb = float((np.mean(p * q) - 1.0) / den) if abs(den) > 1e-12 else float("nan")
    nb = np.linalg.norm(b)
    f_ovl = float(abs(np.vdot(a, b)) ** 2 / (na ** 2 * nb ** 2)) if na > 0 and nb > 0 else float("nan")
    return {
        "rel_l2": float(np.linalg.norm(b - a) / na) if na > 0 else float(np.linalg.norm(b - a)),
        "max_scaled": float(diff.max() / rms) if rms > 0 else float(diff.max()),
        "rel_median": float(np.median(rel)),
        "rel_p99": float(np.quantile(rel, 0.99)),
        "f_xeb": f_xeb,
        "f_ovl": f_ovl,
    }
