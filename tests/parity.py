"""Error measures shared by the GPU parity tests (test-side only).

Potentials: max |f_gpu - f_ref| / max(|f_ref|_inf, eps)   (bar 1e-4)
Map outputs: max_i |T_gpu_i - T_ref_i|_2 / max(|T_ref_i|_2, s_Y)  (bar 1e-3)
  where s_Y = RMS distance of the targets to their mean, so points mapped
  near the origin are measured against the target cloud's scale.
"""
import numpy as np


def pot_err(gpu, ref, eps):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(gpu - ref).max() / max(np.abs(ref).max(), eps))


def gauge_pot_err(f_gpu, g_gpu, f_ref, g_ref, a, b, eps):
    """Potentials are defined up to (f + c, g - c); compare after shifting
    both pairs so that <a, f> = <b, g>."""
    def fix(f, g):
        f = np.asarray(f, np.float64)
        g = np.asarray(g, np.float64)
        c = 0.5 * (a @ f - b @ g)
        return f - c, g + c
    fg, gg = fix(f_gpu, g_gpu)
    fr, gr = fix(f_ref, g_ref)
    return max(pot_err(fg, fr, eps), pot_err(gg, gr, eps))


def map_err(gpu, ref, Y):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    Yd = np.asarray(Y, dtype=np.float64)
    sy = np.sqrt(((Yd - Yd.mean(0)) ** 2).sum(1).mean())
    den = np.maximum(np.linalg.norm(ref, axis=1), sy)
    return float((np.linalg.norm(gpu - ref, axis=1) / den).max())
