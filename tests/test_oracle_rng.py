"""Pins of the oracle's random-number and sampling steps against sources other
than the oracle: rocRAND's Philox4x32-10 (compiled from its public header),
scipy's inverse normal, and closed-form mixture moments."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.special
import scipy.stats

from tests import cases

ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
// reads lines "seed subsequence offset", prints the first 4 words generated
int main() {
  unsigned long long s, q, o;
  while (std::scanf("%llu %llu %llu", &s, &q, &o) == 3) {
    rocrand_device::philox4x32_10_engine e(s, q, o);
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_philox():
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "p.cpp")
    exe = os.path.join(d, "p")
    with open(src, "w") as f:
        f.write(ROCRAND_PROBE)
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    src, "-o", exe], check=True, capture_output=True)

    def run(triples):
        inp = "\n".join(f"{s} {q} {o}" for s, q, o in triples) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                             check=True).stdout
        return np.array([[int(x) for x in ln.split()] for ln in out.strip().splitlines()],
                        dtype=np.uint64)

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(oracle, rocrand_philox):
    # rocRAND engine (seed, subsequence, offset=4k) starts at counter
    # (k lo, k hi, subsequence lo, subsequence hi) with key (seed lo, seed hi).
    rng = np.random.default_rng(5)
    triples, ctrs, keys = [], [], []
    for i in range(300):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        k = int(rng.integers(0, 2**40)) if i % 3 else i
        mol = int(rng.integers(0, 2**32)) if i % 5 else i
        stream = int(rng.integers(0, 4)) if i % 7 == 0 else 0
        triples.append((seed, mol | (stream << 32), 4 * k))
        ctrs.append([k & 0xFFFFFFFF, k >> 32, mol, stream])
        keys.append([seed & 0xFFFFFFFF, seed >> 32])
    ref = rocrand_philox(triples)
    got = np.array([oracle.philox(c, kk) for c, kk in zip(ctrs, keys)], dtype=np.uint64)
    assert np.array_equal(ref, got)


def test_philox_bits_uniform(oracle):
    words = np.array([oracle.philox([k, 0, 7, 0], [123, 456]) for k in range(20000)])
    bits = ((words[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(-1, 128)
    p = bits.mean(0)
    # each bit is Bernoulli(1/2): 20000 draws, sd 0.0035
    assert np.all(np.abs(p - 0.5) < 6 * 0.5 / np.sqrt(20000))
    # adjacent counters are not correlated in word 0
    x = words[:, 0].astype(np.float64)
    r = np.corrcoef(x[:-1], x[1:])[0, 1]
    assert abs(r) < 0.04


def test_norm_inv_matches_scipy(oracle):
    j = np.concatenate([np.arange(0, 200), np.arange(2**24 - 200, 2**24),
                        np.random.default_rng(0).integers(0, 2**24, 3000)])
    u = (j + 0.5) / 2.0**24
    z = np.array([oracle.norm_inv(x) for x in u])
    ref = scipy.special.ndtri(u)
    assert np.all(np.abs(z - ref) <= 2e-14 * np.maximum(1.0, np.abs(ref)))
    assert oracle.norm_inv(0.5) == 0.0
    # the 24-bit uniforms cap |z| at Phi^-1(2^-25)
    assert abs(z).max() == pytest.approx(-scipy.special.ndtri(0.5 / 2**24), rel=1e-12)


def test_alpha_gives_hard_sphere_volume_over_p(oracle):
    """alpha = kappa/(lambda R^2) with lambda = p^(-2/3): a unit-height atom
    Gaussian integrates to (4/3) pi R^3 / p (radial quadrature, not the
    closed form)."""
    R = np.array([1.70, 1.55, 1.52, 1.80], np.float32)
    a = oracle.alpha_from_radius(R, cases.LAMBDA).astype(np.float64)
    for Ri, ai in zip(R.astype(np.float64), a):
        vol, _ = scipy.integrate.quad(lambda r: 4 * np.pi * r * r * np.exp(-ai * r * r),
                                      0, np.inf, epsabs=0, epsrel=1e-12)
        assert vol == pytest.approx(4.0 / 3.0 * np.pi * Ri**3 / 2.7, rel=1e-6)


def test_thresholds(oracle):
    m = cases.config0()[1]
    xyz, alpha = cases.oracle_mol(oracle, m)
    v, Z, thr = oracle.mol_prep(xyz, alpha)
    a = alpha.astype(np.float64)
    assert np.allclose(v, (np.pi / a) ** 1.5, rtol=1e-15)
    assert Z == pytest.approx(v.sum(), rel=1e-15)
    assert np.all(np.diff(thr.astype(np.int64)) >= 0)
    exact = 2.0**32 * np.cumsum(v)[:-1] / Z
    assert np.all(np.abs(thr - exact) < 1.0 + 1e-6)


def test_component_frequencies_chi2(oracle):
    m = cases.config0()[0]
    xyz, alpha = cases.oracle_mol(oracle, m)
    v, Z, _ = oracle.mol_prep(xyz, alpha)
    n = 200000
    _, comp = oracle.sample_points(xyz, alpha, 3, 11, 0, n, return_component=True)
    cnt = np.bincount(comp, minlength=v.size)
    chi2, p = scipy.stats.chisquare(cnt, n * v / Z)
    assert p > 1e-4


def test_mixture_moments_closed_form(oracle):
    """Samples follow q = m/Z: mean sum pi_i c_i and covariance
    sum pi_i (c_i c_i^T + I/(2 alpha_i)) - mu mu^T."""
    m = cases.config0()[1]
    xyz, alpha = cases.oracle_mol(oracle, m)
    c = xyz.astype(np.float64)
    a = alpha.astype(np.float64)
    pi = (np.pi / a) ** 1.5
    pi /= pi.sum()
    mu = (pi[:, None] * c).sum(0)
    cov = (pi[:, None, None] * (c[:, :, None] * c[:, None, :]
                                + np.eye(3)[None] / (2 * a[:, None, None]))).sum(0)
    cov -= np.outer(mu, mu)
    n = 200000
    r = oracle.sample_points(xyz, alpha, 9, 2, 0, n)
    se_mu = np.sqrt(np.diag(cov) / n)
    assert np.all(np.abs(r.mean(0) - mu) < 5 * se_mu)
    emp = np.cov(r.T)
    assert np.allclose(emp, cov, atol=0.03 * np.abs(np.diag(cov)).max())


def test_sample_points_are_counter_indexed(oracle):
    m = cases.small(1, 5)
    xyz, alpha = cases.oracle_mol(oracle, m)
    r_all = oracle.sample_points(xyz, alpha, 42, 77, 0, 300)
    r_tail = oracle.sample_points(xyz, alpha, 42, 77, 200, 100)
    assert np.array_equal(r_all[200:], r_tail)
    r_other = oracle.sample_points(xyz, alpha, 43, 77, 0, 300)
    assert not np.array_equal(r_all, r_other)
