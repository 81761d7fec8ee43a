/*
 * CPU ORACLE — test infrastructure only.
 *
 * Plain, slow, sequential reference for the SMMO workloads run by the GPU
 * library.  Nothing in the product path may link or call this file; only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * Paper: Springer & Masuhara, "DynaSOAr: A Parallel Memory Allocator for
 * Object-oriented Programming on GPUs with Efficient Memory Access",
 * ECOOP 2019 (arXiv 1810.11765).
 *
 * What the oracle computes (Sec. 2.1, "Programming Interface"): a parallel
 * do-all runs a method once on every object of a type that exists when the
 * do-all starts; objects created by the method join afterwards, destroyed
 * objects leave.  Where a block or slot an object lands in is not part of the
 * result, so the oracle keeps plain dense arrays keyed by object id / cell id
 * and no allocator at all.  Every result below is the canonical state: records
 * ordered by id, FP32 values as raw bits.
 *
 * Randomness: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) — written here from that publication; the
 * GPU side has its own independent implementation.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so every FP32 operation is one IEEE-754 rounding in the order written).
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

/* ------------------------------------------------------------------ RNG -- */

/* First output of SplitMix64 seeded with x: advance the state by the golden
 * gamma, then apply the 64-bit finalizer of the publication. */
uint64_t or_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Counter-based draw keyed on (seed, step, object/cell id, stream). */
uint64_t or_ctr(uint64_t seed, uint64_t step, uint64_t id, uint64_t stream)
{
    uint64_t h = or_splitmix64(seed ^ (stream << 56));
    h = or_splitmix64(h ^ step);
    return or_splitmix64(h ^ id);
}

/* Threads the OpenMP loops below use (the CPU-baseline leg reports it). */
int or_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

static float u01(uint64_t h) { return (float)(h >> 40) * (1.0f / 16777216.0f); }
static uint32_t choice(uint64_t h, uint32_t k) { return (uint32_t)((h >> 32) % k); }

/* ------------------------------------------- alloc microbench (one class) --
 * Objects {int32 id, float32 x, float32 v}.  One round r =
 *   do-all 1: v <- v + 0.5*x                       (every live object)
 *   do-all 2: if splitmix64(seed ^ id ^ r) & 1 the object destroys itself and
 *             allocates one replacement with id' = ((r+1) << 18) | (id & 0x3FFFF),
 *             x' = U01(ctr(seed, r+1, id', 0)), v' = U01(ctr(seed, r+1, id', 1)).
 * The replacement is created during do-all 2 and is therefore not visited by
 * it (Sec. 3.1, iteration bitmap).  Arrays hold the live set sorted by id. */

static int cmp_i32_idx(const void* a, const void* b, void* keys)
{
    const int32_t* k = (const int32_t*)keys;
    int32_t x = k[*(const int64_t*)a], y = k[*(const int64_t*)b];
    return (x > y) - (x < y);
}

/* reorder the three arrays by ascending id (ids are unique) */
static void sort_by_id(int64_t n, int32_t* id, float* x, float* v)
{
    int64_t* p = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int32_t* id2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    float* x2 = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    float* v2 = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) p[i] = i;
    qsort_r(p, (size_t)n, sizeof(int64_t), cmp_i32_idx, id);
    for (int64_t i = 0; i < n; ++i) { id2[i] = id[p[i]]; x2[i] = x[p[i]]; v2[i] = v[p[i]]; }
    memcpy(id, id2, sizeof(int32_t) * (size_t)n);
    memcpy(x, x2, sizeof(float) * (size_t)n);
    memcpy(v, v2, sizeof(float) * (size_t)n);
    free(p); free(id2); free(x2); free(v2);
}

/* One round on the live set (n objects, sorted by id on entry and exit).
 * Returns the number of objects that were replaced. */
int64_t or_c1_round(uint64_t seed, uint32_t r, int64_t n, int32_t* id, float* x, float* v)
{
    int64_t replaced = 0;
    for (int64_t i = 0; i < n; ++i)               /* do-all 1 */
        v[i] = v[i] + 0.5f * x[i];
    for (int64_t i = 0; i < n; ++i) {             /* do-all 2 */
        uint64_t h = or_splitmix64(seed ^ (uint64_t)(uint32_t)id[i] ^ (uint64_t)r);
        if (h & 1) {
            int32_t nid = (int32_t)(((uint32_t)(r + 1) << 18) | ((uint32_t)id[i] & 0x3FFFFu));
            id[i] = nid;
            x[i] = u01(or_ctr(seed, r + 1, (uint64_t)(uint32_t)nid, 0));
            v[i] = u01(or_ctr(seed, r + 1, (uint64_t)(uint32_t)nid, 1));
            ++replaced;
        }
    }
    sort_by_id(n, id, x, v);
    return replaced;
}

/* -------------------------------------------------- Life-like grid -------
 * Torus W x H, cell id c = y*W + x.  Cells are static; an Agent {cell, age}
 * exists exactly on each alive cell.  One step =
 *   Cell::plan   next = B3/S23 of the 8 neighbours' current state
 *   Agent::step  if the agent's cell has next = 0 the agent destroys itself,
 *                otherwise age += 1
 *   Cell::commit if the cell was dead and next = 1 a new Agent{c, age 0} is
 *                created; alive <- next
 * alive/age are dense per-cell arrays; age[c] = -1 where no agent lives. */
void or_c2_run(int32_t W, int32_t H, int32_t steps, uint8_t* alive, int32_t* age)
{
    int64_t n = (int64_t)W * H;
    uint8_t* next = (uint8_t*)malloc((size_t)n);
    for (int64_t c = 0; c < n; ++c)
        age[c] = alive[c] ? 0 : -1;
    for (int32_t s = 0; s < steps; ++s) {
        /* every cell's next state depends on the current grid only, and
         * every cell's update on its own entries: both loops split over
         * threads without changing a result */
        #pragma omp parallel for schedule(static)
        for (int32_t y = 0; y < H; ++y)
            for (int32_t x = 0; x < W; ++x) {
                int cnt = 0;
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (dx == 0 && dy == 0) continue;
                        int32_t xx = (x + dx + W) % W, yy = (y + dy + H) % H;
                        cnt += alive[(int64_t)yy * W + xx];
                    }
                uint8_t a = alive[(int64_t)y * W + x];
                next[(int64_t)y * W + x] = (uint8_t)(a ? (cnt == 2 || cnt == 3) : (cnt == 3));
            }
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < n; ++c) {
            if (alive[c]) {                        /* agent lives here */
                if (next[c]) age[c] += 1;
                else age[c] = -1;                  /* destroyed */
            } else if (next[c]) {
                age[c] = 0;                        /* born */
            }
            alive[c] = next[c];
        }
    }
    free(next);
}

/* ---------------------------------------------- Predator-prey (Wa-Tor) ----
 * Torus W x H.  kind[c] in {0 empty, 1 fish, 2 shark}; age, energy per cell.
 * Neighbour order N, E, S, W = (x, y-1), (x+1, y), (x, y+1), (x-1, y).
 * Conflicts for a target cell are won by the lowest current position.
 * Step s (1-based):
 *  F1 every fish: age += 1; among empty neighbours pick
 *     cand[(ctr(seed,s,pos,1) >> 32) % ncand]; claim it.
 *  F2 every fish whose claim won moves; if its age >= fish_breed it leaves a
 *     new fish (age 0) behind and resets its age to 0.
 *  S1 every shark: age += 1; candidates = fish neighbours, else empty
 *     neighbours; pick with stream 2; claim.
 *  S2 every shark that exists when S2 starts: if its claim won it moves, eats
 *     the fish on the target (energy += eat_gain) and, if age >= shark_breed,
 *     leaves a new shark (age 0, energy shark_e0) behind and resets its age;
 *     then energy -= 1 and at 0 it dies.
 * counts (optional, 6 per step): fish and sharks after the step, fish eaten,
 * sharks starved, fish born, sharks born. */
void or_c3_run(int32_t W, int32_t H, uint64_t seed, int32_t steps,
               int32_t fish_breed, int32_t shark_breed, int32_t eat_gain, int32_t shark_e0,
               uint8_t* kind, int32_t* age, int32_t* energy, int64_t* counts)
{
    int64_t n = (int64_t)W * H;
    int32_t* claim = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* want = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t* phase = (uint8_t*)malloc((size_t)n);   /* snapshot of who takes part */
    for (int64_t c = 0; c < n; ++c) claim[c] = INT32_MAX;

    for (int32_t s = 1; s <= steps; ++s) {
        int64_t eaten = 0, starved = 0, fborn = 0, sborn = 0;
        /* F1 */
        for (int64_t c = 0; c < n; ++c) phase[c] = (kind[c] == 1);
        for (int64_t c = 0; c < n; ++c) {
            if (!phase[c]) continue;
            int32_t x = (int32_t)(c % W), y = (int32_t)(c / W);
            int64_t nb[4] = { (int64_t)((y - 1 + H) % H) * W + x, (int64_t)y * W + (x + 1) % W,
                              (int64_t)((y + 1) % H) * W + x, (int64_t)y * W + (x - 1 + W) % W };
            age[c] += 1;
            int64_t cand[4]; int nc = 0;
            for (int k = 0; k < 4; ++k) if (kind[nb[k]] == 0) cand[nc++] = nb[k];
            want[c] = -1;
            if (nc) {
                int64_t t = cand[choice(or_ctr(seed, (uint64_t)s, (uint64_t)c, 1), (uint32_t)nc)];
                want[c] = (int32_t)t;
                if ((int32_t)c < claim[t]) claim[t] = (int32_t)c;
            }
        }
        /* F2: reads only want/claim of phase-start fish; targets were empty at
         * phase start, so a move never lands on a cell another fish leaves. */
        for (int64_t c = 0; c < n; ++c) {
            if (!phase[c] || want[c] < 0) continue;
            int64_t t = want[c];
            if (claim[t] != (int32_t)c) continue;
            kind[t] = 1; age[t] = age[c]; energy[t] = 0;
            if (age[t] >= fish_breed) { age[t] = 0; kind[c] = 1; age[c] = 0; energy[c] = 0; ++fborn; }
            else { kind[c] = 0; age[c] = 0; energy[c] = 0; }
        }
        for (int64_t c = 0; c < n; ++c) claim[c] = INT32_MAX;
        /* S1 */
        for (int64_t c = 0; c < n; ++c) phase[c] = (kind[c] == 2);
        for (int64_t c = 0; c < n; ++c) {
            if (!phase[c]) continue;
            int32_t x = (int32_t)(c % W), y = (int32_t)(c / W);
            int64_t nb[4] = { (int64_t)((y - 1 + H) % H) * W + x, (int64_t)y * W + (x + 1) % W,
                              (int64_t)((y + 1) % H) * W + x, (int64_t)y * W + (x - 1 + W) % W };
            age[c] += 1;
            int64_t cand[4]; int nc = 0;
            for (int k = 0; k < 4; ++k) if (kind[nb[k]] == 1) cand[nc++] = nb[k];
            if (!nc) for (int k = 0; k < 4; ++k) if (kind[nb[k]] == 0) cand[nc++] = nb[k];
            want[c] = -1;
            if (nc) {
                int64_t t = cand[choice(or_ctr(seed, (uint64_t)s, (uint64_t)c, 2), (uint32_t)nc)];
                want[c] = (int32_t)t;
                if ((int32_t)c < claim[t]) claim[t] = (int32_t)c;
            }
        }
        /* S2: sharks present at S2 start are exactly phase[]; a target holds
         * either nothing or a fish (never a shark), and no target equals the
         * origin of another shark, so the sequential order is irrelevant. */
        for (int64_t c = 0; c < n; ++c) {
            if (!phase[c]) continue;
            int64_t pos = c;
            int32_t a = age[c], e = energy[c];
            if (want[c] >= 0 && claim[want[c]] == (int32_t)c) {
                int64_t t = want[c];
                if (kind[t] == 1) { e += eat_gain; ++eaten; }
                kind[t] = 2;
                if (a >= shark_breed) { a = 0; kind[c] = 2; age[c] = 0; energy[c] = shark_e0; phase[c] = 0; ++sborn; }
                else { kind[c] = 0; age[c] = 0; energy[c] = 0; }
                pos = t;
                phase[t] = 0;    /* t now holds this shark; it was not a phase-start shark */
            }
            e -= 1;
            if (e <= 0) { kind[pos] = 0; age[pos] = 0; energy[pos] = 0; ++starved; }
            else { age[pos] = a; energy[pos] = e; }
        }
        for (int64_t c = 0; c < n; ++c) claim[c] = INT32_MAX;
        if (counts) {
            int64_t nf = 0, ns = 0;
            for (int64_t c = 0; c < n; ++c) { nf += kind[c] == 1; ns += kind[c] == 2; }
            int64_t* q = counts + 6 * (int64_t)(s - 1);
            q[0] = nf; q[1] = ns; q[2] = eaten; q[3] = starved; q[4] = fborn; q[5] = sborn;
        }
    }
    free(claim); free(want); free(phase);
}

/* ------------------------------------------------- N-body with merging ----
 * Bodies {x, y, vx, vy, m} in FP32, addressed by id (ascending ids on entry
 * and exit).  One step (Sec. 1, n-body with collisions; the force is the
 * gravitational all-pairs sum of the API example, divided by the body's own
 * mass so that it is an acceleration):
 *  (M) pairs with sqrtf(dx*dx + dy*dy) < merge_dist are joined; every
 *      connected component keeps its lowest id, which keeps its position and
 *      takes m' = sum m_k and v' = (sum m_k v_k) / m', both sums running over
 *      the component in ascending id; every other member is destroyed.
 *  (F) a_i = sum over j != i in ascending id of s*(dx, dy), dx = x_j - x_i,
 *      d2 = dx*dx + dy*dy, s = (G*m_j) / (d2*sqrtf(d2)); v += a*dt.
 *  (P) x += v*dt.
 * Returns the number of survivors (arrays compacted in place). */
static int64_t uf_find(int64_t* p, int64_t i)
{
    while (p[i] != i) { p[i] = p[p[i]]; i = p[i]; }
    return i;
}

/* Phases (F) and (P) on the n bodies of a merged state (ascending id):
 * a_i = sum over j != i in ascending id of s*(dx, dy), dx = x_j - x_i,
 * d2 = dx*dx + dy*dy, s = (G*m_j) / (d2*sqrtf(d2)); v += a*dt; x += v*dt.
 * The bodies' sums are independent; each runs over j in ascending order. */
static void c4_force_move(int64_t n, float* x, float* y, float* vx, float* vy, const float* m,
                          float G, float dt)
{
    float* ax = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    float* ay = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float sx = 0.0f, sy = 0.0f;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            float dx = x[j] - x[i], dy = y[j] - y[i];
            float d2 = dx * dx + dy * dy;
            float s = (G * m[j]) / (d2 * sqrtf(d2));
            sx = sx + s * dx;
            sy = sy + s * dy;
        }
        ax[i] = sx; ay[i] = sy;
    }
    for (int64_t i = 0; i < n; ++i) {
        vx[i] = vx[i] + ax[i] * dt;
        vy[i] = vy[i] + ay[i] * dt;
        x[i] = x[i] + vx[i] * dt;
        y[i] = y[i] + vy[i] * dt;
    }
    free(ax); free(ay);
}

int64_t or_c4_step(int64_t n, int32_t* id, float* x, float* y, float* vx, float* vy, float* m,
                   float G, float dt, float merge_dist, int64_t* npairs_out)
{
    /* (M) brute-force pair search, union-find with the smallest index as root */
    int64_t* par = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) par[i] = i;
    int64_t npairs = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            float dx = x[j] - x[i], dy = y[j] - y[i];
            float d = sqrtf(dx * dx + dy * dy);
            if (d < merge_dist) {
                int64_t a = uf_find(par, i), b = uf_find(par, j);
                if (a < b) par[b] = a; else if (b < a) par[a] = b;
                ++npairs;
            }
        }
    if (npairs_out) *npairs_out = npairs;
    /* accumulate each component at its root, members visited in ascending id */
    float* ms = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    float* px = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    float* py = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    uint8_t* seen = (uint8_t*)calloc((size_t)(n ? n : 1), 1);
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = uf_find(par, i);
        if (!seen[r]) { seen[r] = 1; ms[r] = m[i]; px[r] = m[i] * vx[i]; py[r] = m[i] * vy[i]; }
        else { ms[r] = ms[r] + m[i]; px[r] = px[r] + m[i] * vx[i]; py[r] = py[r] + m[i] * vy[i]; }
    }
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (uf_find(par, i) != i) continue;         /* destroyed */
        int comp = 0;
        for (int64_t j = i + 1; j < n && !comp; ++j) comp = (uf_find(par, j) == i);
        id[k] = id[i]; x[k] = x[i]; y[k] = y[i];
        if (comp) { m[k] = ms[i]; vx[k] = px[i] / ms[i]; vy[k] = py[i] / ms[i]; }
        else { m[k] = m[i]; vx[k] = vx[i]; vy[k] = vy[i]; }
        ++k;
    }
    n = k;
    free(par); free(ms); free(px); free(py); free(seen);

    c4_force_move(n, x, y, vx, vy, m, G, dt);
    return n;
}

/* Acceleration of selected bodies only (same sum as phase F), for checking a
 * large state one body at a time. */
void or_c4_accel(int64_t n, const float* x, const float* y, const float* m, float G,
                 int64_t nsel, const int64_t* sel, float* ax, float* ay)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nsel; ++q) {
        int64_t i = sel[q];
        float sx = 0.0f, sy = 0.0f;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            float dx = x[j] - x[i], dy = y[j] - y[i];
            float d2 = dx * dx + dy * dy;
            float s = (G * m[j]) / (d2 * sqrtf(d2));
            sx = sx + s * dx;
            sy = sy + s * dy;
        }
        ax[q] = sx; ay[q] = sy;
    }
}

/* Merge phase (M) alone, for checking a large state: the same rule as in
 * or_c4_step, with candidate pairs taken from a uniform grid of cell edge
 * `cell` >= merge_dist (two bodies closer than merge_dist are in the same or
 * in adjacent cells), each candidate decided by the same float test.
 * Returns the survivor count; arrays are compacted in place. */
typedef struct { int64_t cx, cy, i; } or_cellrec;
static int cmp_cellrec(const void* a, const void* b)
{
    const or_cellrec* p = (const or_cellrec*)a; const or_cellrec* q = (const or_cellrec*)b;
    if (p->cx != q->cx) return p->cx < q->cx ? -1 : 1;
    if (p->cy != q->cy) return p->cy < q->cy ? -1 : 1;
    return (p->i > q->i) - (p->i < q->i);
}

int64_t or_c4_merge_grid(int64_t n, int32_t* id, float* x, float* y, float* vx, float* vy, float* m,
                         float merge_dist, double cell, int64_t* npairs_out)
{
    or_cellrec* rec = (or_cellrec*)malloc(sizeof(or_cellrec) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        rec[i].cx = (int64_t)floor((double)x[i] / cell);
        rec[i].cy = (int64_t)floor((double)y[i] / cell);
        rec[i].i = i;
    }
    qsort(rec, (size_t)n, sizeof(or_cellrec), cmp_cellrec);
    int64_t* par = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; ++i) par[i] = i;
    int64_t npairs = 0;
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t dx = -1; dx <= 1; ++dx)
            for (int64_t dy = -1; dy <= 1; ++dy) {
                or_cellrec key = { rec[a].cx + dx, rec[a].cy + dy, -1 };
                /* first record of that cell */
                int64_t lo = 0, hi = n;
                while (lo < hi) {
                    int64_t mid = (lo + hi) / 2;
                    if (cmp_cellrec(&rec[mid], &key) < 0) lo = mid + 1; else hi = mid;
                }
                for (int64_t b = lo; b < n && rec[b].cx == key.cx && rec[b].cy == key.cy; ++b) {
                    int64_t i = rec[a].i, j = rec[b].i;
                    if (j <= i) continue;              /* each pair once, i < j */
                    float ddx = x[j] - x[i], ddy = y[j] - y[i];
                    float d = sqrtf(ddx * ddx + ddy * ddy);
                    if (d < merge_dist) {
                        int64_t ra = uf_find(par, i), rb = uf_find(par, j);
                        if (ra < rb) par[rb] = ra; else if (rb < ra) par[ra] = rb;
                        ++npairs;
                    }
                }
            }
    }
    if (npairs_out) *npairs_out = npairs;
    float* ms = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    float* px = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    float* py = (float*)malloc(sizeof(float) * (size_t)(n ? n : 1));
    int32_t* cnt = (int32_t*)calloc((size_t)(n ? n : 1), sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = uf_find(par, i);
        if (cnt[r]++ == 0) { ms[r] = m[i]; px[r] = m[i] * vx[i]; py[r] = m[i] * vy[i]; }
        else { ms[r] = ms[r] + m[i]; px[r] = px[r] + m[i] * vx[i]; py[r] = py[r] + m[i] * vy[i]; }
    }
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (uf_find(par, i) != i) continue;
        id[k] = id[i]; x[k] = x[i]; y[k] = y[i];
        if (cnt[i] > 1) { m[k] = ms[i]; vx[k] = px[i] / ms[i]; vy[k] = py[i] / ms[i]; }
        else { m[k] = m[i]; vx[k] = vx[i]; vy[k] = vy[i]; }
        ++k;
    }
    free(rec); free(par); free(ms); free(px); free(py); free(cnt);
    return k;
}

/* One whole step (M), (F), (P) with the merge's candidate pairs taken from the
 * grid of or_c4_merge_grid: the same result as or_c4_step (the grid only
 * narrows which pairs are tested), at a cost that large states can afford. */
int64_t or_c4_step_grid(int64_t n, int32_t* id, float* x, float* y, float* vx, float* vy, float* m,
                        float G, float dt, float merge_dist, double cell, int64_t* npairs_out)
{
    n = or_c4_merge_grid(n, id, x, y, vx, vy, m, merge_dist, cell, npairs_out);
    c4_force_move(n, x, y, vx, vy, m, G, dt);
    return n;
}
