// Compile-time lattice data for the device code.
//
// D2Q9: velocities and weights of Eq. 5, transform M0 of Eq. 15 (rows rho, e,
// eps, jx, qx, jy, qy, pxx, pxy).  D3Q19: velocities and weights of Eq. 6 and
// the orthogonal polynomial basis of d'Humieres et al. (2002) in that
// velocity order.  Loops over these tables are fully unrolled so that every
// entry becomes an immediate and the zero entries vanish.
#pragma once

namespace lbm {

template <int Q>
struct Lattice;

template <>
struct Lattice<9> {
    static constexpr int dim = 2;
    static constexpr int jrow[3] = {3, 5, -1};
    static constexpr int jnorm = 6;  // sum_k c_kx^2
    __host__ __device__ static constexpr int cx(int k) {
        constexpr int v[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        return v[k];
    }
    __host__ __device__ static constexpr int cy(int k) {
        constexpr int v[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        return v[k];
    }
    __host__ __device__ static constexpr int cz(int) { return 0; }
    __host__ __device__ static constexpr int c(int k, int a) { return a == 0 ? cx(k) : (a == 1 ? cy(k) : 0); }
    __host__ __device__ static constexpr double w(int k) {
        return k == 0 ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int k) {
        constexpr int v[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        return v[k];
    }
    __host__ __device__ static constexpr int M(int i, int k) {
        constexpr int m[9][9] = {
            {1, 1, 1, 1, 1, 1, 1, 1, 1},
            {-4, -1, -1, -1, -1, 2, 2, 2, 2},
            {4, -2, -2, -2, -2, 1, 1, 1, 1},
            {0, 1, 0, -1, 0, 1, -1, -1, 1},
            {0, -2, 0, 2, 0, 1, -1, -1, 1},
            {0, 0, 1, 0, -1, 1, 1, -1, -1},
            {0, 0, -2, 0, 2, 1, 1, -1, -1},
            {0, 1, -1, 1, -1, 0, 0, 0, 0},
            {0, 0, 0, 0, 0, 1, -1, 1, -1}};
        return m[i][k];
    }
    // row norms diag(M M^T)
    __host__ __device__ static constexpr int N(int i) {
        constexpr int v[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};
        return v[i];
    }
};

template <>
struct Lattice<19> {
    static constexpr int dim = 3;
    static constexpr int jrow[3] = {3, 5, 7};
    static constexpr int jnorm = 10;
    __host__ __device__ static constexpr int cx(int k) {
        constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0};
        return v[k];
    }
    __host__ __device__ static constexpr int cy(int k) {
        constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        return v[k];
    }
    __host__ __device__ static constexpr int cz(int k) {
        constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
        return v[k];
    }
    __host__ __device__ static constexpr int c(int k, int a) { return a == 0 ? cx(k) : (a == 1 ? cy(k) : cz(k)); }
    __host__ __device__ static constexpr double w(int k) {
        return k == 0 ? 1.0 / 3.0 : (k < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }
    // basis row i at velocity k (polynomials of c)
    __host__ __device__ static constexpr int M(int i, int k) {
        const int x = cx(k), y = cy(k), z = cz(k);
        const int c2 = x * x + y * y + z * z;
        switch (i) {
            case 0: return 1;
            case 1: return 19 * c2 - 30;
            case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
            case 3: return x;
            case 4: return (5 * c2 - 9) * x;
            case 5: return y;
            case 6: return (5 * c2 - 9) * y;
            case 7: return z;
            case 8: return (5 * c2 - 9) * z;
            case 9: return 3 * x * x - c2;
            case 10: return (3 * c2 - 5) * (3 * x * x - c2);
            case 11: return y * y - z * z;
            case 12: return (3 * c2 - 5) * (y * y - z * z);
            case 13: return x * y;
            case 14: return y * z;
            case 15: return x * z;
            case 16: return (y * y - z * z) * x;
            case 17: return (z * z - x * x) * y;
            default: return (x * x - y * y) * z;
        }
    }
    __host__ __device__ static constexpr int N(int i) {
        int acc = 0;
        for (int k = 0; k < 19; ++k) acc += M(i, k) * M(i, k);
        return acc;
    }
};

// symmetric tensor slot of (a, b): (xx, yy, zz, xy, yz, xz)
__host__ __device__ constexpr int sym(int a, int b) {
    return a == b ? a : ((a + b == 1) ? 3 : ((a + b == 3) ? 4 : 5));
}

}  // namespace lbm
