"""The FP32 rounding floor of one right-hand side, measured with an
independent single-precision library pipeline (scipy.fft in float32/
complex64, the same truncation, products, projection and damping).  It sets
the FP32 parity bound where the arithmetic itself cannot reach 1e-5: the
physical-space FP32 products carry white rounding noise that the k-weighting
of the divergence amplifies at high k."""
import numpy as np


def rhs_single_precision(uh, n, eps, s=1.5, m_cut=None):
    import scipy.fft as sf

    K = (n - 1) // 3
    m = n / 3.0 if m_cut is None else m_cut
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kh = np.arange(n // 2 + 1)
    KZ, KY, KX = np.meshgrid(k1, k1, kh, indexing="ij")
    T = (np.abs(KZ) <= K) & (np.abs(KY) <= K) & (KX <= K)
    u = uh.astype(np.complex64) * T
    up = sf.irfftn(u, s=(n, n, n), axes=(-3, -2, -1), norm="forward", workers=8).astype(np.float32)
    B = {}
    for i in range(3):
        for j in range(i, 3):
            B[(i, j)] = B[(j, i)] = sf.rfftn(up[i] * up[j], axes=(-3, -2, -1), norm="forward",
                                            workers=8).astype(np.complex64) * T
    kv = [KX.astype(np.float32), KY.astype(np.float32), KZ.astype(np.float32)]
    b = [-1j * sum(kv[j] * B[(i, j)] for j in range(3)) for i in range(3)]
    k2 = (KX ** 2 + KY ** 2 + KZ ** 2).astype(np.float32)
    k2s = np.where(k2 > 0, k2, 1)
    kb = sum(kv[j] * b[j] for j in range(3))
    c = [b[i] - kv[i] * kb / k2s for i in range(3)]
    rate = (eps * k2.astype(np.float64) ** s * (np.sqrt(k2) > m)).astype(np.float32)
    return np.stack([(c[i] - rate * u[i]) * T for i in range(3)]).astype(np.complex128)


def fp32_floor(uh, n, ref, eps, s=1.5, m_cut=None):
    F = rhs_single_precision(uh, n, eps, s, m_cut)
    return float(np.linalg.norm(F - ref) / np.linalg.norm(ref))
