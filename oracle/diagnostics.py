"""Macroscopic fields, conserved sums and the energy spectrum (the oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

fields      -- stage (c) of the step (Sec. II / III C): the Landau-frame
               eps, beta and T^{mu nu} of the streamed populations, i.e. the
               macroscopic variables the next step computes (Sec. V records
               them every step).
conserved   -- sum over the lattice of T^{00}, T^{0x}, T^{0y} of the stored
               populations (streaming preserves each plane's sum).
spectrum    -- Sec. IV: E(k) is the kinetic energy per wave-number magnitude.
               Reading (the printed definition mixes a density, an angular
               average and a derivative): shell sum
                   E(k_b) = sum_{round(|k|) = k_b} 1/2 |beta_hat(k)|^2,
               beta_hat = DFT(beta) / (nx ny), integer k in [-n/2, n/2)^2.
               The paper's spectral energy density, half the squared velocity
               amplitude averaged over the directions of k, is on the lattice
               the shell sum divided by the shell's number of wave vectors
               (shell_modes).
               Enstrophy (Sec. IV, vorticity w = curl v):
                   Z = 1/2 sum_k |w_hat(k)|^2,
                   w_hat = i (2 pi kx / nx) beta_hat_y - i (2 pi ky / ny) beta_hat_x.
filtered_velocity -- Sec. V: the recorded velocities have the driven band
               removed in Fourier space; their lattice average speed is the
               quantity the forcing amplitude is tuned by.
spectrum_average -- appendix on the minimum simulation time: time average of
               sampled spectra and the paper's error estimate.
"""
import numpy as np

from . import rlbm


def fields(F, st, cfl=1.0):
    """(eps, beta_x, beta_y, T6) of the streamed populations.

    T6 stacks T^{00}, T^{0x}, T^{0y}, T^{xx}, T^{xy}, T^{yy}.
    """
    Fs = rlbm.stream(F, st, cfl)
    T, _ = rlbm.moments(Fs, st)
    eps, u = rlbm.landau(T)
    beta = u[1:] / u[0]
    T6 = np.stack([T[0, 0], T[0, 1], T[0, 2], T[1, 1], T[1, 2], T[2, 2]])
    return eps, beta[0], beta[1], T6


def conserved(F, st):
    T, _ = rlbm.moments(F, st)
    return np.array([T[0, 0].sum(), T[0, 1].sum(), T[0, 2].sum()])


def spectrum(beta_x, beta_y, nbins):
    """Shell-summed kinetic energy spectrum and enstrophy (reading above)."""
    ny, nx = beta_x.shape
    bx = np.fft.fft2(beta_x) / (nx * ny)
    by = np.fft.fft2(beta_y) / (nx * ny)
    kx = np.fft.fftfreq(nx, 1.0 / nx)          # integers, [-n/2, n/2)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")
    e = 0.5 * (np.abs(bx) ** 2 + np.abs(by) ** 2)
    shell = np.rint(np.sqrt(KX ** 2 + KY ** 2)).astype(np.int64)
    Ek = np.zeros(nbins)
    keep = shell < nbins
    np.add.at(Ek, shell[keep], e[keep])
    w = 1j * (2 * np.pi * KX / nx) * by - 1j * (2 * np.pi * KY / ny) * bx
    Z = 0.5 * (np.abs(w) ** 2).sum()
    return Ek, Z


def shell_modes(nx, ny, nbins):
    """Number of integer wave vectors k (DFT numbering, as in ``spectrum``)
    with round(|k|) = b, for b = 0 .. nbins-1: dividing a shell sum by it
    gives the average over the directions of k (Sec. IV)."""
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")
    shell = np.rint(np.sqrt(KX ** 2 + KY ** 2)).astype(np.int64).ravel()
    return np.bincount(shell[shell < nbins], minlength=nbins)[:nbins]


def filtered_velocity(beta_x, beta_y, k_lo, k_hi):
    """Velocity with the driven band removed, and its average speed.

    Sec. V: every Fourier mode of beta with k_lo <= |k| <= k_hi (integer k in
    [-n/2, n/2)^2, the same shell test as the forcing modes) is set to zero and
    the field transformed back; the average fluid velocity is the lattice
    mean of |beta_filtered|.
    """
    ny, nx = beta_x.shape
    kx = np.fft.fftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")
    k2 = KX ** 2 + KY ** 2
    keep = ~((k2 >= k_lo * k_lo) & (k2 <= k_hi * k_hi))
    fx = np.fft.ifft2(np.fft.fft2(beta_x) * keep).real
    fy = np.fft.ifft2(np.fft.fft2(beta_y) * keep).real
    return fx, fy, float(np.mean(np.sqrt(fx ** 2 + fy ** 2)))


def spectrum_average(samples):
    """Mean spectrum and error estimate of M spectra sampled a decorrelation
    interval apart (appendix on the minimum simulation time): the error of
    bin k is the sample average of sqrt(<E(k)>^2 - E_i(k)^2), read with the
    magnitude of the difference under the root (it can be negative)."""
    samples = np.asarray(samples, dtype=np.float64)
    mean = samples.mean(axis=0)
    err = np.sqrt(np.abs(mean[None, :] ** 2 - samples ** 2)).mean(axis=0)
    return mean, err
