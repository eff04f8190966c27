"""Newton march over dG(k) slabs with the solver of this package, and the learned
initial guess (a project extension; Sec. 3 solves every slab by Newton's method,
which needs a starting point).

NewtonMarch solves F(X) = 0 slab after slab: each Newton step assembles J(X) on
every level (the caller's problem object, on the host), copies the values into
the device matrices (the sparsity never changes), runs vanka_setup and
gmres_solve for J C = -F, and damps the update by backtracking (lambda in
{1, 1/2, 1/4, 1/8, 1/16}, first with ||F(X + lambda C)|| <= (1 - 1e-4 lambda)
||F(X)||).  Newton stops at ||F|| < tol (absolute); GMRES at
max(rtol ||F||, atol).

Guesses for slab n from the two previous solutions:
  * ExtrapolationGuess: the previous slab's time polynomial evaluated at the new
    Radau nodes (HIP kernel);
  * LearnedGuess: that extrapolation plus the averaged patch corrections of the
    BF16 network (feature gather, forward pass and DoF averaging are HIP
    kernels; training runs the library's gradient and Adam kernels);
  * JudgedGuess: the learned guess with the extrapolation as fallback, judged by
    the slab residual: both candidates are evaluated with F of Eq. 2.2 (the same
    residual Newton stops on) and Newton starts from the one with the smaller
    ||F||, whose residual it reuses.

The problem object provides initial_slab(), hierarchy(X) (levels with J, P, R,
cell_dofs, colours), residual(X, X_prev, n), E (the extrapolation matrix) and
fine.mesh (n, n_K, n_cells, cell_dofs()).
"""
import time

import numpy as np
import torch

from . import MLP, Solver, dof_entries, upload_level

DAMPING = (1.0, 0.5, 0.25, 0.125, 0.0625)


class NewtonMarch:
    def __init__(self, problem, device="cuda:0", prec="f32", tol=1e-8, rtol=1e-8, atol=1e-10, nu=(2, 2),
                 max_newton=20, omega=0.7):
        self.pr, self.dev = problem, device
        self.tol, self.rtol, self.atol, self.nu, self.max_newton, self.omega = tol, rtol, atol, nu, max_newton, omega
        levels = problem.hierarchy(problem.initial_slab())
        self.levels = [upload_level(L, device) for L in levels]
        self.S = Solver(self.levels)
        self.S.vk_set_workspace(prec, 30, device=device)
        self.S.vanka_setup(omega)
        self.n = levels[-1].J.shape[0]
        self.b = torch.zeros(self.n, dtype=torch.float64, device=device)
        self.c = torch.zeros_like(self.b)

    def close(self):
        self.S.close()

    def _load_jacobians(self, X):
        for lv, L in zip(self.levels, self.pr.hierarchy(X)):
            lv["J"]["val"].copy_(torch.from_numpy(L.J.data))

    def solve_slab(self, X0, X_prev, n, F0=None):
        """Newton iteration of slab n from X0 (F0: its residual, if already evaluated); returns
        (X, stats)."""
        t_asm = t_gpu = t_res = 0.0
        X = np.array(X0, dtype=np.float64, copy=True)
        t0 = time.perf_counter()
        F = self.pr.residual(X, X_prev, n) if F0 is None else F0
        t_res += time.perf_counter() - t0
        nrm = float(np.linalg.norm(F))
        st = {"F0": nrm, "newton": 0, "gmres": 0, "hist": [nrm]}
        while nrm >= self.tol and st["newton"] < self.max_newton:
            t0 = time.perf_counter()
            self._load_jacobians(X)
            t1 = time.perf_counter()
            self.b.copy_(torch.from_numpy(-F))
            self.c.zero_()
            self.S.vanka_setup(self.omega)
            its, _, _, _ = self.S.gmres_solve(self.b, self.c, rtol=self.rtol, atol=self.atol, nu_pre=self.nu[0],
                                              nu_post=self.nu[1])
            C = self.c.cpu().numpy()
            t2 = time.perf_counter()
            t_asm += t1 - t0
            t_gpu += t2 - t1
            st["gmres"] += its
            for lam in DAMPING:
                Xt = X + lam * C
                Ft = self.pr.residual(Xt, X_prev, n)
                nt = float(np.linalg.norm(Ft))
                if nt <= (1.0 - 1e-4 * lam) * nrm:
                    break
            t_res += time.perf_counter() - t2
            X, F, nrm = Xt, Ft, nt
            st["newton"] += 1
            st["hist"].append(nrm)
        st.update(t_assembly=t_asm, t_solve=t_gpu, t_residual=t_res, converged=nrm < self.tol)
        return X, st


class ExtrapolationGuess:
    """Fallback guess: the previous slab's Lagrange time polynomial at the new nodes."""

    def __init__(self, problem, device="cuda:0", kernels=None):
        self.pr, self.dev = problem, device
        self.k = kernels if kernels is not None else MLP(1, 1, 1, 1, 1, device=device)
        m = problem.fine.mesh
        self.X = torch.zeros(m.n, dtype=torch.float64, device=device)
        self.out = torch.zeros_like(self.X)

    def extrapolate_device(self, X_prev_dev, out):
        self.k.slab_extrapolate(self.pr.E, X_prev_dev, out)

    def __call__(self, n, X_prev2, X_prev):
        self.X.copy_(torch.from_numpy(np.asarray(X_prev)))
        self.extrapolate_device(self.X, self.out)
        return self.out.cpu().numpy()


class LearnedGuess:
    """Extrapolation plus the BF16 network's averaged patch corrections."""

    def __init__(self, problem, width, n_hidden, device="cuda:0", max_batch=4096):
        self.pr, self.dev = problem, device
        m = problem.fine.mesh
        self.n_K, self.n_cells, self.n = m.n_K, m.n_cells, m.n
        self.net = MLP(2 * m.n_K, width, n_hidden, m.n_K, max(max_batch, m.n_cells), device=device)
        self.ext = ExtrapolationGuess(problem, device, kernels=self.net)
        cd = m.cell_dofs()
        self.cell_dofs_h = cd
        self.cell_dofs = torch.from_numpy(cd).to(device)
        ptr, lst = dof_entries(cd, m.n)
        self.dof_ptr = torch.from_numpy(ptr).to(device)
        self.dof_list = torch.from_numpy(lst).to(device)
        self.X1 = torch.zeros(m.n, dtype=torch.float64, device=device)
        self.X2 = torch.zeros_like(self.X1)
        self.base = torch.zeros_like(self.X1)
        self.prev_base = torch.zeros_like(self.X1)
        self.out = torch.zeros_like(self.X1)
        self.feat = torch.zeros((m.n_cells, 2 * m.n_K), dtype=torch.bfloat16, device=device)
        self.pred = torch.zeros((m.n_cells, m.n_K), dtype=torch.float32, device=device)
        self.losses = []

    # ---- normalisation statistics (host, once, from the training slabs) -----------------------
    def _stats(self, slabs):
        cd = self.cell_dofs_h
        ext = self.pr.extrapolate
        ins, tg = [], []
        for n in range(2, len(slabs)):
            x2, x1 = slabs[n - 2], slabs[n - 1]
            ins.append(np.concatenate([(x1 - x2)[cd], (x1 - ext(x2))[cd]], axis=1))
            tg.append((slabs[n] - ext(x1))[cd])
        ins = np.concatenate(ins)
        tg = np.concatenate(tg)
        to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.dev)
        sd_in = np.maximum(ins.std(axis=0), 1e-30)
        sd_out = np.maximum(tg.std(axis=0), 1e-30)
        self.in_mean, self.in_inv = to(ins.mean(axis=0)), to(1.0 / sd_in)
        self.out_mean, self.out_sd, self.out_inv = to(tg.mean(axis=0)), to(sd_out), to(1.0 / sd_out)

    def build_dataset(self, slabs):
        """Features and targets of slabs 2..N from the solutions X_0..X_N (host arrays):
        inputs from (X_{n-2}, X_{n-1}) on each cell patch, target X_n - extrapolate(X_{n-1})."""
        self._stats(slabs)
        S = len(slabs) - 2
        feats = torch.empty((S * self.n_cells, 2 * self.n_K), dtype=torch.bfloat16, device=self.dev)
        targs = torch.empty((S * self.n_cells, self.n_K), dtype=torch.float32, device=self.dev)
        Xd = [torch.from_numpy(np.asarray(s)).to(self.dev) for s in slabs]
        prev_base = torch.empty_like(self.base)
        for i in range(S):
            n = i + 2
            sl = slice(i * self.n_cells, (i + 1) * self.n_cells)
            self.ext.extrapolate_device(Xd[n - 2], prev_base)
            self.ext.extrapolate_device(Xd[n - 1], self.base)
            self.net.patch_features(self.cell_dofs, Xd[n - 2], Xd[n - 1], prev_base, self.in_mean, self.in_inv,
                                    feats[sl])
            self.net.patch_targets(self.cell_dofs, Xd[n], self.base, self.out_mean, self.out_inv, targs[sl])
        return feats, targs

    def fit(self, slabs, params0, orders, batch=512, lr=1e-3, lr_min=1e-5):
        """Train on the slab solutions with Adam; orders[e] is epoch e's sample permutation
        (int32, host).  The learning rate follows a cosine from lr to lr_min over the epochs."""
        feats, targs = self.build_dataset(slabs)
        n_s = feats.shape[0]
        assert orders.shape[1] == n_s
        self.net.set_params(torch.from_numpy(params0).to(self.dev))
        self.losses = []
        E = orders.shape[0]
        t0 = time.perf_counter()
        for e in range(E):
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * e / E))
            order = torch.from_numpy(orders[e]).to(self.dev)
            acc = torch.zeros(1, dtype=torch.float32, device=self.dev)
            nb = 0
            for s in range(0, n_s - batch + 1, batch):
                loss, _ = self.net.gradient(feats, targs, rows=order[s:s + batch], want_grad=False)
                self.net.adam(float(rate))
                acc += loss
                nb += 1
            self.losses.append(float(acc.item()) / max(nb, 1))
        self.train_seconds = time.perf_counter() - t0
        return self.losses

    def __call__(self, n, X_prev2, X_prev):
        self.X2.copy_(torch.from_numpy(np.asarray(X_prev2)))
        self.X1.copy_(torch.from_numpy(np.asarray(X_prev)))
        self.ext.extrapolate_device(self.X2, self.prev_base)
        self.ext.extrapolate_device(self.X1, self.base)
        self.net.patch_features(self.cell_dofs, self.X2, self.X1, self.prev_base, self.in_mean, self.in_inv,
                                self.feat)
        self.net.forward(self.feat, out=self.pred)
        self.net.patch_average(self.dof_ptr, self.dof_list, self.n_K, self.pred, self.out_mean, self.out_sd,
                               self.base, self.out)
        return self.out.cpu().numpy()


class JudgedGuess:
    """The learned guess with the plain extrapolation as fallback, the slab residual as judge: both
    candidates are evaluated with the problem's F (Eq. 2.2, the residual Newton iterates on; it is
    assembled by the caller's problem object on the host, as in every Newton step), and the one with
    the smaller ||F|| is returned.  `last_F` keeps its residual for the first Newton step and
    `choices` counts the picks."""

    def __init__(self, learned, fallback, problem):
        self.learned, self.fallback, self.pr = learned, fallback, problem
        self.last_F = None
        self.choices = {"learned": 0, "extrapolation": 0}

    def __call__(self, n, X_prev2, X_prev):
        Xl = self.learned(n, X_prev2, X_prev)
        Xe = self.fallback(n, X_prev2, X_prev)
        Fl = self.pr.residual(Xl, X_prev, n)
        Fe = self.pr.residual(Xe, X_prev, n)
        if np.linalg.norm(Fl) <= np.linalg.norm(Fe):
            self.choices["learned"] += 1
            self.last_F = Fl
            return Xl
        self.choices["extrapolation"] += 1
        self.last_F = Fe
        return Xe


def march(nm, first, last, slabs, guess):
    """Slabs first..last with NewtonMarch nm; slabs holds X_0..X_{first-1} and is extended.
    Returns the per-slab statistics."""
    stats = []
    for n in range(first, last + 1):
        prev = slabs[n - 1]
        prev2 = slabs[n - 2] if n >= 2 else slabs[n - 1]
        t0 = time.perf_counter()
        X0 = guess(n, prev2, prev)
        F0 = getattr(guess, "last_F", None)
        t1 = time.perf_counter()
        X, st = nm.solve_slab(X0, prev, n, F0=F0)
        st["t_guess"] = t1 - t0
        st["t_total"] = time.perf_counter() - t0
        slabs.append(X)
        stats.append(st)
    return stats
